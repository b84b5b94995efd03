"""Pins of the oracle's weight-window grid planes (windows checked where a
flight reaches an interior plane of a regular grid over the outer box, tie
order census < surface < grid plane < collision): deterministic void beams
up and down (the plane each particle stops on, its time, the split there,
the particle that starts on a plane moving off it), a plane that coincides
with a geometry surface (the surface event wins), unbiased tallies against
the analog run, and invalid grids.  CPU only."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from oracle import oracle as O
from paper_2409_04668_amd import workloads as W


def _flat_mlp():
    """y = 0 everywhere (all weights and biases zero)."""
    return np.zeros(M.n_params(5, 64), np.float32)


def _void_box(direction, grid=(4, 2, 2), boxes=False):
    p = W._base(1)
    p["outer_lo"] = np.zeros(3)
    p["outer_hi"] = np.full(3, 20.0)
    p["sigma_t"] = np.array([[0.0]])
    p["sigma_s"] = np.array([[[0.0]]])
    p["source"] = dict(kind="point", lo=np.full(3, 10.0), hi=np.full(3, 10.0), t0=0.0, t1=0.0,
                       isotropic=False, dir=np.asarray(direction, float), group=0)
    p["mesh"] = dict(lo=np.array([0.0, 0.0, 0.0, 0.0]), hi=np.array([20.0, 20.0, 20.0, 40.0]),
                     n=np.array([4, 2, 2, 4], np.int32), per_group=False)
    p["census"] = np.array([40.0])
    # w_T = exp(log 0.25 - 0) = 1/4: a unit weight splits into four at its first check
    p["ww"] = dict(params=_flat_mlp(), hidden=64, logk=math.log(0.25), ratio=5.0, n_max=10,
                   grid=grid)
    if boxes:
        p["box_lo"] = np.array([[15.0, 0.0, 0.0]])
        p["box_hi"] = np.array([[20.0, 20.0, 20.0]])
        p["box_mat"] = np.array([0], np.int32)
    return p


@pytest.mark.parametrize("direction,plane", [((1.0, 0.0, 0.0), 15.0), ((-1.0, 0.0, 0.0), 5.0)])
def test_void_beam_stops_on_the_next_interior_plane(direction, plane):
    """From (10, 10, 10), itself on the planes x = 10, y = 10, z = 10 of a
    4 x 2 x 2 grid over [0, 20]^3: the beam moves off x = 10, stops on the next
    interior plane 5 cm away (at t = 5), splits into four there, and the four
    copies, standing on that plane, reach the outer face without another stop."""
    p = _void_box(direction)
    n = 200
    r = O.OracleRun(p)
    tr, _ = r.run(n, seed=3, trace_cap=100000)
    c = r.counters
    assert c["ww_plane"] == n and c["split"] == 3 * n and c["leak"] == 4 * n
    wp = tr[tr["type"] == O.EV["ww_plane"]]
    assert len(wp) == n
    assert np.all(wp["x"] == plane) and np.all(wp["y"] == 10.0) and np.all(wp["z"] == 10.0)
    assert np.all(wp["t"] == 5.0) and np.all(wp["aux"] == 5.0)
    assert r.wsum["leak"] == float(n) and r.wsum["source"] == float(n)


def test_grid_plane_on_a_surface_yields_to_the_surface_event():
    """The box face x = 15 lies on the grid plane x = 15: the flight ends in
    a surface event there (tie order), and the windows are checked after it."""
    p = _void_box((1.0, 0.0, 0.0), boxes=True)
    n = 200
    r = O.run(p, n, seed=4)
    c = r.counters
    assert c["ww_plane"] == 0 and c["split"] == 3 * n and c["surface"] >= 5 * n


def test_grid_off_is_the_plain_window_run():
    """Without a grid the run is the earlier one, bit for bit."""
    p = _void_box((1.0, 0.0, 0.0))
    q = dict(p)
    q["ww"] = dict(p["ww"], grid=None)
    a = O.run(q, 300, seed=5)
    b = O.run(dict(q), 300, seed=5)
    assert a.counters["ww_plane"] == 0
    assert np.array_equal(a.tally_sum, b.tally_sum)
    assert a.counters["split"] == 0       # no check ever happens in the void without a grid


def _ramp_mlp(slope):
    prm = np.zeros(M.n_params(5, 64), np.float32)
    prm[0] = 1.0
    prm[64 * 5] = 1.0
    prm[64 * 5 + 64] = 1.0
    prm[64 * 5 + 64 + 64 * 64 + 64] = slope
    prm[-1] = -slope
    return prm


def test_grid_windows_stay_unbiased_against_analog():
    p = W._base(1)
    p["outer_lo"] = np.zeros(3)
    p["outer_hi"] = np.full(3, 20.0)
    p["sigma_t"] = np.array([[0.3]])
    p["sigma_s"] = np.array([[[0.2]]])
    p["source"] = dict(kind="point", lo=np.full(3, 10.0), hi=np.full(3, 10.0), t0=0.0, t1=0.0,
                       isotropic=True, dir=np.array([1.0, 0.0, 0.0]), group=0)
    p["mesh"] = dict(lo=np.zeros(4), hi=np.array([20.0, 20.0, 20.0, 40.0]),
                     n=np.array([10, 1, 1, 4], np.int32), per_group=False)
    p["census"] = np.array([40.0])
    N = 40000
    ra = O.run(p, N, seed=21)
    q = dict(p)
    q["ww"] = dict(params=_ramp_mlp(2.0), hidden=64, logk=0.0, ratio=5.0, n_max=10,
                   ymin=-1.5, ymax=1.5, grid=(10, 4, 4))
    rw = O.run(q, N, seed=22)
    assert rw.counters["ww_plane"] > N and rw.counters["split"] > 1000
    ma, sa = ra.mesh_stats()
    mw, sw = rw.mesh_stats()
    ok = (sa > 0) & (sw > 0)
    z = np.abs(ma - mw)[ok] / np.sqrt(sa[ok] ** 2 + sw[ok] ** 2)
    assert ok.sum() >= 30 and np.max(z) < 4.5 and np.mean(z < 3) > 0.9
    ws = rw.wsum
    assert abs(ws["source"] + ws["gain"] - ws["loss"] - ws["leak"] - ws["absorb"] - ws["time_end"]) \
        <= 1e-9 * ws["source"]


@pytest.mark.parametrize("grid", [(4, 0, 2), (0, 0, -1)])
def test_invalid_grids_rejected(grid):
    p = _void_box((1.0, 0.0, 0.0), grid=grid)
    with pytest.raises(O.OracleError):
        O.run(p, 10, seed=1)


def test_grid_without_windows_rejected():
    p = _void_box((1.0, 0.0, 0.0))
    p["ww"] = None
    r = O.OracleRun(p)
    r.P.s.ww_grid_n = (type(r.P.s.ww_grid_n))(2, 2, 2)
    with pytest.raises(O.OracleError):
        r.run(10, seed=1)
