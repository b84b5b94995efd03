"""Pins of the oracle's surface-current tally (weight of every flight that
crosses the plane x[axis] = pos, binned by side, group, time and the mesh
bins of the other two axes): a void beam (every particle crosses once, in a
known bin), a beam through a pure absorber (transmission e^{-Sigma h}), an
isotropic point source in a pure absorber (partial current E2(Sigma h)/2, no
return current), the exact per-history identity J+ - J- = leakage through the
far face in a scattering slab, and a brute-force re-scoring of every flight
segment of event traces in a two-group problem with a partial mesh.  CPU
only."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import oracle as O
from paper_2409_04668_amd import workloads as W


def _open_box(sig_t, sig_s, half=50.0, t_end=100.0, nt=10, n=(10, 4, 4), isotropic=False):
    p = W._base(1)
    p["outer_lo"] = np.full(3, -half)
    p["outer_hi"] = np.full(3, half)
    p["sigma_t"] = np.array([[sig_t]])
    p["sigma_s"] = np.array([[[sig_s]]])
    p["source"] = dict(kind="point", lo=np.zeros(3), hi=np.zeros(3), t0=0.0, t1=0.0,
                       isotropic=isotropic, dir=np.array([1.0, 0.0, 0.0]), group=0)
    p["mesh"] = dict(lo=np.array([-half, -half, -half, 0.0]), hi=np.array([half, half, half, t_end]),
                     n=np.array([n[0], n[1], n[2], nt], np.int32), per_group=False)
    p["census"] = np.array([t_end])
    p["n_batches"] = 4
    return p


def _surf(r):
    """(J+, J-) per source particle, summed over all bins."""
    mean, _ = r.mesh_stats("surface")
    half = mean.size // 2
    return mean[:half].sum(), mean[half:].sum()


def test_void_beam_crosses_once_in_a_known_bin():
    p = _open_box(0.0, 0.0)
    p["surface_tally"] = dict(axis=0, pos=20.5)
    n = 1000
    r = O.run(p, n, seed=3)
    assert r.counters["surf_cross"] == n
    s = r.surf_sum.reshape(2, 1, 10, 4, 4)        # side, group, t, z, y
    # crossing at y = z = 0 (bins 2 of 4 over [-50, 50]) at t = 20.5 (bin 2 of 10)
    assert s[0, 0, 2, 2, 2] == float(n)
    assert s.sum() == float(n)
    # a plane behind the beam is never crossed
    q = dict(p, surface_tally=dict(axis=0, pos=-10.0))
    assert O.run(q, n, seed=3).counters["surf_cross"] == 0


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_beam_transmission_through_pure_absorber(axis):
    p = _open_box(1.0, 0.0, half=10.0, t_end=20.0, nt=4, n=(2, 2, 2))
    d = np.zeros(3)
    d[axis] = 1.0
    p["source"]["dir"] = d
    p["surface_tally"] = dict(axis=axis, pos=1.5)
    n = 100_000
    r = O.run(p, n, seed=5 + axis)
    jp, jm = _surf(r)
    e = math.exp(-1.5)
    assert jm == 0.0
    assert abs(jp - e) < 4 * math.sqrt(e * (1 - e) / n)


def test_isotropic_point_source_partial_current_is_e2_over_2():
    """Pure absorber, plane at distance h: the uncollided partial current
    through the (effectively infinite) plane is E2(Sigma h)/2; nothing comes
    back."""
    sig, h = 1.0, 1.0
    p = _open_box(sig, 0.0, half=30.0, t_end=40.0, nt=4, n=(1, 6, 6), isotropic=True)
    p["surface_tally"] = dict(axis=0, pos=h)
    n = 200_000
    r = O.run(p, n, seed=7)
    jp, jm = _surf(r)
    e = special.expn(2, sig * h) / 2.0
    assert jm == 0.0
    assert abs(jp - e) < 4 * math.sqrt(e * (1 - e) / n)
    # crossings spread over the y-z bins symmetrically
    s = r.surf_sum.reshape(2, 1, 4, 6, 6)[0].sum(axis=(0, 1))
    assert np.allclose(s, s.T, rtol=0.2, atol=50)


def test_net_current_equals_leakage_through_far_face():
    """Scattering slab (c = 1, reflective y and z faces, vacuum x faces), a
    late end time so that every particle leaks: a particle from x = 0 that
    leaks through +x crossed the plane x = h once more upward than downward,
    one that leaks through -x as often each way.  Summed over histories,
    J+ - J- equals the weight leaked through +x exactly."""
    p = _open_box(1.0, 1.0, half=4.0, t_end=1.0e5, nt=1, n=(1, 1, 1), isotropic=True)
    p["bc"] = np.array([0, 0, 1, 1, 1, 1], np.int32)
    p["surface_tally"] = dict(axis=0, pos=1.25)
    n = 5000
    r = O.run(p, n, seed=11)
    assert r.counters["time_end"] == 0
    up = r.surf_sum[0]
    down = r.surf_sum[1]
    assert up - down == r.leak[1]
    assert r.counters["surf_cross"] > 2 * n


def _two_group_box():
    p = W._base(2)
    p["outer_lo"] = np.zeros(3)
    p["outer_hi"] = np.full(3, 10.0)
    p["box_lo"] = np.array([[4.0, 0.0, 0.0]])
    p["box_hi"] = np.array([[7.0, 10.0, 10.0]])
    p["box_mat"] = np.array([1], np.int32)
    p["sigma_t"] = np.array([[0.4, 0.6], [1.5, 2.0]])
    p["sigma_s"] = np.array([[[0.2, 0.1], [0.0, 0.5]], [[1.0, 0.3], [0.0, 1.8]]])
    p["speed"] = np.array([2.0, 0.5])
    p["source"] = dict(kind="box", lo=np.array([1.0, 1.0, 1.0]), hi=np.array([9.0, 9.0, 9.0]),
                       t0=0.0, t1=3.0, isotropic=True, dir=np.array([1.0, 0.0, 0.0]), group=0)
    # the mesh covers only part of the plane and of the time range
    p["mesh"] = dict(lo=np.array([2.0, 0.0, 1.0, 0.0]), hi=np.array([9.0, 10.0, 8.0, 8.0]),
                     n=np.array([7, 4, 5, 6], np.int32), per_group=True)
    p["census"] = np.array([5.0, 12.0])
    p["n_batches"] = 3
    p["surface_tally"] = dict(axis=1, pos=6.5)
    return p


def test_surface_tally_brute_force_from_trace():
    """Every flight segment rebuilt from consecutive trace records of a
    particle (the earlier record holds the flight's start state, the later
    one its length) and re-scored by hand."""
    p = _two_group_box()
    r = O.OracleRun(p)
    tr, _ = r.run(8000, seed=13, trace_cap=2_000_000)
    assert len(tr) < 2_000_000
    tr = tr[np.lexsort((tr["seq"], tr["tag"], tr["hist"]))]
    m = p["mesh"]
    lo, hi, n = m["lo"], m["hi"], m["n"]
    idelta = [1.0 / ((hi[a] - lo[a]) / n[a]) for a in range(4)]
    want = np.zeros(2 * 2 * n[3] * n[0] * n[2])
    a, b1, b2 = 1, 0, 2
    c = 6.5
    crossings = outside = 0
    for i in range(1, len(tr)):
        e0, e1 = tr[i - 1], tr[i]
        if e0["hist"] != e1["hist"] or e0["tag"] != e1["tag"]:
            continue
        p0 = (e0["x"], e0["y"], e0["z"])
        u = (e0["ux"], e0["uy"], e0["uz"])
        d = e1["aux"]
        if u[a] == 0.0:
            continue
        sx = (c - p0[a]) * (1.0 / u[a])
        if not (sx > 0.0 and sx <= d):
            continue
        crossings += 1
        f1 = math.floor((p0[b1] + u[b1] * sx - lo[b1]) * idelta[b1])
        f2 = math.floor((p0[b2] + u[b2] * sx - lo[b2]) * idelta[b2])
        ft = math.floor((e0["t"] + sx / p["speed"][e0["g"]] - lo[3]) * idelta[3])
        if not (0 <= f1 < n[b1] and 0 <= f2 < n[b2] and 0 <= ft < n[3]):
            outside += 1
            continue
        side = 0 if u[a] > 0.0 else 1
        b = (((side * 2 + e0["g"]) * n[3] + ft) * n[b2] + f2) * n[b1] + f1
        want[b] += e0["w"]
    assert crossings > 1000 and outside > 100
    assert r.counters["surf_cross"] == crossings - outside
    np.testing.assert_allclose(r.surf_sum, want, rtol=1e-12, atol=1e-300)
    # both sides and both groups are scored
    s = r.surf_sum.reshape(2, 2, -1).sum(axis=2)
    assert np.all(s > 0)


def test_invalid_surface_axis_rejected():
    p = _open_box(1.0, 0.0)
    p["surface_tally"] = dict(axis=3, pos=0.0)
    with pytest.raises(O.OracleError):
        O.run(p, 10, seed=1)
