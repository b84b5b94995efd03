"""GPU parity of the mesh walk's edge cases against the oracle: segments that
start outside the mesh in space and in time, enter, leave and re-enter it (a
partial mesh inside the geometry); beams along the diagonal from a mesh
corner, so that the three spatial axes cross their edges at the same distance
on every piece; a beam lying in a mesh plane; a beam that starts on a plane
moving down.  Each case runs under the history, event and hybrid schedules
(the analog kernels) and with a weight-window map (the window kernels, whose
walk recomputes its crossing steps): one particle per history bit-identical,
split particles to 1e-12, tally sums to 1e-10, counters exact."""
import math

import numpy as np
import pytest

from paper_2409_04668_amd import workloads as W

from gpu_util import assert_close_sums, assert_counters, assert_traces_equal, full_parity, run_pair
from test_gpu_parity import ramp_mlp

pytestmark = pytest.mark.gpu

SCHEDS = ["history", "event", "hybrid"]


def _opt(sched, tile=None):
    from paper_2409_04668_amd import mcdc as mc
    return mc.make_options({"history": mc.SCHED_HISTORY, "event": mc.SCHED_EVENT,
                            "hybrid": mc.SCHED_HYBRID}[sched], tile=tile)


def _partial_mesh_box():
    """Scattering box [0,10]^3; the mesh covers [2,8]x[3,7]x[1.5,9] and the
    time range [1,6] of a run that starts at t in [0,2] and ends at 12."""
    p = W._base(1)
    p["outer_lo"] = np.zeros(3)
    p["outer_hi"] = np.full(3, 10.0)
    p["sigma_t"] = np.array([[0.3]])
    p["sigma_s"] = np.array([[[0.2]]])
    p["source"] = dict(kind="box", lo=np.full(3, 0.5), hi=np.full(3, 9.5), t0=0.0, t1=2.0,
                       isotropic=True, dir=np.array([1.0, 0.0, 0.0]), group=0)
    p["mesh"] = dict(lo=np.array([2.0, 3.0, 1.5, 1.0]), hi=np.array([8.0, 7.0, 9.0, 6.0]),
                     n=np.array([6, 8, 5, 10], np.int32), per_group=False)
    p["census"] = np.array([12.0])
    p["n_batches"] = 4
    return p


def _beam(point, direction, sigma_t=0.05):
    """Thin scatterer in [0,10]^3 with a 1 cm mesh over [2,8]^3 and 1 s time
    bins; a point source with a fixed direction."""
    p = W._base(1)
    p["outer_lo"] = np.zeros(3)
    p["outer_hi"] = np.full(3, 10.0)
    p["sigma_t"] = np.array([[sigma_t]])
    p["sigma_s"] = np.array([[[sigma_t / 2]]])
    d = np.asarray(direction, float)
    p["source"] = dict(kind="point", lo=np.asarray(point, float), hi=np.asarray(point, float),
                       t0=0.0, t1=0.0, isotropic=False, dir=d / math.sqrt(float(d @ d)), group=0)
    p["mesh"] = dict(lo=np.array([2.0, 2.0, 2.0, 0.0]), hi=np.array([8.0, 8.0, 8.0, 20.0]),
                     n=np.array([6, 6, 6, 20], np.int32), per_group=False)
    p["census"] = np.array([20.0])
    p["n_batches"] = 4
    return p


BEAMS = {
    "diagonal_up_from_corner": ((5.0, 5.0, 5.0), (1.0, 1.0, 1.0)),
    "diagonal_down_from_corner": ((5.0, 5.0, 5.0), (-1.0, -1.0, -1.0)),
    "diagonal_entering_from_outside": ((0.5, 0.5, 0.5), (1.0, 1.0, 1.0)),
    "in_a_mesh_plane": ((5.0, 4.0, 3.0), (0.0, 1.0, 0.0)),
    "down_from_a_plane": ((3.0, 5.5, 6.5), (-1.0, 0.0, 0.0)),
}


@pytest.mark.parametrize("sched", SCHEDS)
def test_walk_partial_mesh_enter_leave(sched):
    tile = ([1, 1, 0, 2, 0], [3, 4, 3, 5, 1]) if sched != "event" else None
    gp, orc = full_parity(_partial_mesh_box(), 3000, seed=301, trace_cap=400000,
                          options=_opt(sched, tile))
    assert orc.counters["piece"] > 5000 and orc.counters["time_end"] > 50
    gp.close()


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("beam", sorted(BEAMS))
def test_walk_beams_with_ties(beam, sched):
    point, direction = BEAMS[beam]
    gp, orc = full_parity(_beam(point, direction), 1500, seed=302, trace_cap=200000,
                          options=_opt(sched))
    assert orc.counters["piece"] > 1500
    gp.close()


@pytest.mark.parametrize("sched", ["history", "event", "hybrid"])
def test_walk_partial_mesh_with_window_map(sched):
    """The weight-window kernels (split particles, crossing steps recomputed
    in the walk)."""
    p = _partial_mesh_box()
    p["ww"] = dict(params=ramp_mlp(-1.5, noise_seed=7), hidden=64, logk=0.3, ratio=5.0, n_max=10,
                   map=(10, 10, 10, 6))
    tile = ([1, 1, 0, 2, 0], [3, 4, 3, 5, 1]) if sched != "event" else None
    gp, orc, tg, to, hg, ho = run_pair(p, 1500, 303, trace_cap=600000, options=_opt(sched, tile))
    assert_traces_equal(tg[0], to[0])
    np.testing.assert_allclose(hg[0], ho[0], rtol=1e-12, atol=1e-300)
    s, s2 = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")
    assert_counters(gp.counters(), orc)
    assert orc.counters["split"] > 10
    gp.close()
