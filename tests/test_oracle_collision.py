"""Pins of the oracle's collision-estimator mesh tally (w / Sigma_t per
collision, scored in the bin of the collision point; its expectation is the
bin's track length): pulsed infinite-medium decay in one group (analog and
implicit capture) and in three groups (matrix exponential), a brute-force
re-scoring of collision events from the event trace, and agreement with the
track-length estimator on the duct problem.  CPU only."""
import math

import numpy as np
import pytest
from scipy import linalg

from oracle import oracle as O
from paper_2409_04668_amd import workloads as W


@pytest.mark.parametrize("implicit", [False, True])
def test_collision_estimator_pulsed_infinite_medium(implicit):
    sig_t, sig_s, v = 1.0, 0.6, 2.0
    sig_a = sig_t - sig_s
    p = W.infinite_medium(sig_t, [[sig_s]], [v], half=5.0, t_end=4.0, nt=8, implicit=implicit)
    p["w_cut"] = 0.05
    p["collision_tally"] = True
    N = 40000
    r = O.run(p, N, seed=19 + implicit)
    mean, se = r.mesh_stats("collision")
    edges = np.linspace(0, 4.0, 9)
    exp_ = (np.exp(-v * sig_a * edges[:-1]) - np.exp(-v * sig_a * edges[1:])) / sig_a
    assert np.all(np.abs(mean - exp_) < 4 * se), (mean, exp_, se)
    # the track-length tally of the same run is untouched by the extra tally
    q = dict(p, collision_tally=False)
    r2 = O.run(q, N, seed=19 + implicit)
    assert np.array_equal(r.tally_sum, r2.tally_sum)


def test_collision_estimator_multigroup_infinite_medium():
    st = np.array([0.5, 0.8, 1.0])
    ss = np.array([[0.3, 0.0, 0.0],
                   [0.2, 0.4, 0.0],
                   [0.1, 0.3, 0.5]])
    v = np.array([1.0, 3.0, 10.0])
    p = W.infinite_medium(st, ss, v, half=5.0, t_end=2.0, nt=4, src_group=2)
    p["collision_tally"] = True
    N = 40000
    r = O.run(p, N, seed=23)
    mean, se = r.mesh_stats("collision")
    mean = mean.reshape(3, 4)
    se = se.reshape(3, 4)
    A = ss.T @ np.diag(v) - np.diag(v * st)
    Z = np.zeros((3, 3))

    def F(T):  # int_0^T exp(A s) ds
        M = linalg.expm(np.block([[A, np.eye(3)], [Z, Z]]) * T)
        return M[:3, 3:]

    n0 = np.array([0.0, 0.0, 1.0])
    edges = np.linspace(0, 2.0, 5)
    for it in range(4):
        exp_ = v * ((F(edges[it + 1]) - F(edges[it])) @ n0)
        assert np.all(np.abs(mean[:, it] - exp_) < 4 * se[:, it] + 1e-12), (it, mean[:, it], exp_)


def _two_material_box():
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
    # the mesh covers only part of the box and of the time range
    p["mesh"] = dict(lo=np.array([2.0, 0.0, 1.0, 0.0]), hi=np.array([9.0, 10.0, 8.0, 8.0]),
                     n=np.array([7, 4, 5, 6], np.int32), per_group=False)
    p["census"] = np.array([5.0, 12.0])
    p["n_batches"] = 3
    p["collision_tally"] = True
    return p


def test_collision_estimator_brute_force_from_trace():
    """Every analog collision (scatter or absorption record: position, time
    and the unchanged weight at the collision) re-scored by hand."""
    p = _two_material_box()
    r = O.OracleRun(p)
    tr, _ = r.run(3000, seed=29, trace_cap=400000)
    assert len(tr) < 400000
    col = tr[(tr["type"] == O.EV["scatter"]) | (tr["type"] == O.EV["absorb"])]
    assert len(col) > 1000
    lo = p["mesh"]["lo"]
    hi = p["mesh"]["hi"]
    n = p["mesh"]["n"]
    want = np.zeros(int(np.prod(n)))
    outside = 0
    for e in col:
        pt = (e["x"], e["y"], e["z"], e["t"])
        idx = []
        for a in range(4):
            f = math.floor((pt[a] - lo[a]) * (1.0 / ((hi[a] - lo[a]) / n[a])))
            idx.append(f)
        if any(i < 0 or i >= n[a] for a, i in enumerate(idx)):
            outside += 1
            continue
        sig = p["sigma_t"][1 if e["cell"] == 0 else 0][0]
        b = ((idx[3] * n[2] + idx[2]) * n[1] + idx[1]) * n[0] + idx[0]
        want[b] += e["w"] / sig
    assert outside > 100
    np.testing.assert_allclose(r.col_sum, want, rtol=1e-12, atol=1e-300)
    # batch sums of squares are consistent with the batches' totals
    assert np.all(r.col_sumsq >= r.col_sum ** 2 / 3000 * (1 - 1e-12))


def test_collision_and_track_length_estimators_agree():
    p = W.config2()
    p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    p["collision_tally"] = True
    N = 40000
    r = O.run(p, N, seed=31)
    mt, st_ = r.mesh_stats("track")
    mc, sc = r.mesh_stats("collision")
    ok = (st_ > 0) & (sc > 0)
    assert ok.sum() > 50
    z = np.abs(mt - mc)[ok] / np.sqrt(st_[ok] ** 2 + sc[ok] ** 2)
    assert np.mean(z < 3) > 0.95 and np.max(z) < 5
    # totals over the mesh agree closely (the same histories drive both)
    assert abs(mc.sum() - mt.sum()) < 4 * math.sqrt((sc ** 2).sum() + (st_ ** 2).sum())
