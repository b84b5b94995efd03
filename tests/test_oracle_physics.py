"""Pins of the oracle's transport loop against results the mathematics fixes:
uncollided transmission exp(-Sigma_t L) and (1/2) E2(Sigma_t L), the uncollided
space-time flux of a pulsed plane source (numerical quadrature), pulsed
infinite-medium decay exp(-v Sigma_a t) (analog and implicit capture), its
multigroup form via a matrix exponential, the analog collision-count law,
exponential flight lengths, hand-checked deterministic trajectories, a brute
force re-scoring of event traces, and weight/path conservation.  CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate, linalg, special, stats

from oracle import oracle as O
from paper_2409_04668_amd import workloads as W

BIG = 1e9


def _beam_slab(sigma_t, L, isotropic):
    p = W.slab_problem(sigma_t=sigma_t, c=0.0, length=L, t_end=BIG, nx=10, nt=1, detector=None)
    p["source"]["isotropic"] = isotropic
    p["source"]["dir"] = np.array([1.0, 0.0, 0.0])
    return p


def _binom_ok(k, n, p, nsig=3.5):
    return abs(k - n * p) <= nsig * math.sqrt(n * p * (1 - p))


def test_uncollided_slab_transmission_beam():
    N = 100000
    r = O.run(_beam_slab(1.0, 2.0, isotropic=False), N, seed=5)
    transmitted = int(round(r.leak[1]))
    assert r.leak[0] == 0.0                         # a +x beam never leaks backwards
    assert _binom_ok(transmitted, N, math.exp(-2.0))
    assert r.counters["absorb"] + transmitted == N


def test_uncollided_slab_transmission_isotropic():
    N = 200000
    r = O.run(_beam_slab(1.0, 1.0, isotropic=True), N, seed=6)
    # half the source (mu < 0) leaks through x=0 at birth
    transmitted = int(round(r.leak[1]))
    assert _binom_ok(int(round(r.leak[0])), N, 0.5)
    assert _binom_ok(transmitted, N, 0.5 * special.expn(2, 1.0))


def test_uncollided_space_time_flux():
    """Pure absorber (c=0), pulsed isotropic plane source at x=0: expected
    track length per source particle in bin [x1,x2]x[t1,t2] is
    int_{t1}^{t2} v e^{-Sigma v t} (1/2) |[x1/(vt), x2/(vt)] cap (0,1]| dt."""
    sig, v = 1.0, 1.0
    p = W.slab_problem(sigma_t=sig, c=0.0, length=10.0, t_end=10.0, nx=10, nt=5, v=v,
                       detector=None)
    N = 200000
    r = O.run(p, N, seed=8)
    mean, se = r.mesh_stats()
    mean = mean.reshape(5, 10)
    se = se.reshape(5, 10)

    def expected(x1, x2, t1, t2):
        def f(t):
            a = min(1.0, x1 / (v * t)) if t > 0 else 0.0
            b = min(1.0, x2 / (v * t)) if t > 0 else 0.0
            return v * math.exp(-sig * v * t) * 0.5 * max(b - a, 0.0)
        pts = [x for x in (x1 / v, x2 / v) if t1 < x < t2]
        return integrate.quad(f, t1, t2, points=pts or None, limit=200, epsabs=1e-13)[0]

    checked = 0
    for it in range(5):
        for ix in range(10):
            e = expected(ix * 1.0, ix + 1.0, it * 2.0, it * 2.0 + 2.0)
            if e < 1e-4:
                assert mean[it, ix] < 1e-3
                continue
            assert abs(mean[it, ix] - e) < 4 * se[it, ix] + 1e-12, (it, ix, mean[it, ix], e, se[it, ix])
            checked += 1
    assert checked >= 10


@pytest.mark.parametrize("implicit", [False, True])
def test_pulsed_infinite_medium_decay(implicit):
    sig_t, sig_s, v = 1.0, 0.6, 2.0
    sig_a = sig_t - sig_s
    p = W.infinite_medium(sig_t, [[sig_s]], [v], half=5.0, t_end=4.0, nt=8, implicit=implicit)
    p["w_cut"] = 0.05
    N = 40000
    r = O.run(p, N, seed=9 + implicit)
    mean, se = r.mesh_stats()
    edges = np.linspace(0, 4.0, 9)
    exp_ = (np.exp(-v * sig_a * edges[:-1]) - np.exp(-v * sig_a * edges[1:])) / sig_a
    assert np.all(np.abs(mean - exp_) < 4 * se), (mean, exp_, se)
    # surviving population at the end time: weight reaching t_end
    surv = r.wsum["time_end"] / N
    pop = math.exp(-v * sig_a * 4.0)
    if not implicit:
        assert _binom_ok(r.counters["time_end"], N, pop)
    else:
        assert abs(surv - pop) < 0.05 * pop + 4 * math.sqrt(pop / N)


def test_multigroup_infinite_medium():
    st = np.array([0.5, 0.8, 1.0])
    ss = np.array([[0.3, 0.0, 0.0],
                   [0.2, 0.4, 0.0],
                   [0.1, 0.3, 0.5]])
    v = np.array([1.0, 3.0, 10.0])
    p = W.infinite_medium(st, ss, v, half=5.0, t_end=2.0, nt=4, src_group=2)
    N = 40000
    r = O.run(p, N, seed=13)
    mean, se = r.mesh_stats()
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
        pop_int = (F(edges[it + 1]) - F(edges[it])) @ n0
        exp_ = v * pop_int
        assert np.all(np.abs(mean[:, it] - exp_) < 4 * se[:, it] + 1e-12), (it, mean[:, it], exp_)


def test_analog_collision_law():
    c = 0.7
    p = W.infinite_medium(1.0, [[c]], [1.0], half=5.0, t_end=1e6, nt=1)
    N = 50000
    r = O.run(p, N, seed=17)
    cnt = r.counters
    assert cnt["absorb"] == N and cnt["time_end"] == 0
    mean_coll = cnt["collision"] / N
    sd = math.sqrt(c) / (1 - c)                 # geometric on {1,2,...} with p = 1-c
    assert abs(mean_coll - 1 / (1 - c)) < 4 * sd / math.sqrt(N)


def test_flight_lengths_are_exponential():
    # beam in a large pure absorber: absorption depth ~ Exp(Sigma_t)
    sig = 0.7
    p = W.infinite_medium(sig, [[0.0]], [1.0], half=500.0, t_end=1e6, nt=1)
    p["source"]["isotropic"] = False
    p["source"]["dir"] = np.array([1.0, 0.0, 0.0])
    r = O.OracleRun(p)
    tr, _ = r.run(20000, seed=19, trace_cap=50000)
    x = tr[tr["type"] == O.EV["absorb"]]["x"]
    assert x.size == 20000
    assert stats.kstest(x, "expon", args=(0, 1 / sig)).pvalue > 1e-3


def _void_problem():
    p = W._base(1)
    p["outer_lo"] = np.zeros(3)
    p["outer_hi"] = np.full(3, 10.0)
    p["box_lo"] = np.array([[2.0, 0.0, 0.0]])
    p["box_hi"] = np.array([[4.0, 10.0, 10.0]])
    p["box_mat"] = np.array([1], np.int32)
    p["background_mat"] = 0
    p["sigma_t"] = np.zeros((2, 1))
    p["sigma_s"] = np.zeros((2, 1, 1))
    p["speed"] = np.array([2.0])
    p["source"] = dict(kind="point", lo=np.array([1.0, 5.0, 5.0]), hi=np.array([1.0, 5.0, 5.0]),
                       t0=0.0, t1=0.0, isotropic=False, dir=np.array([1.0, 0.0, 0.0]), group=0)
    p["mesh"] = dict(lo=np.array([0.0, 0.0, 0.0, 0.0]), hi=np.array([10.0, 10.0, 10.0, 10.0]),
                     n=np.array([10, 1, 1, 10], np.int32), per_group=False)
    p["census"] = np.array([1.0, 100.0])
    p["n_batches"] = 1
    return p


def test_hand_checked_void_trajectory():
    """Void cells, fixed +x direction, speed 2: surface at x=2 (t=0.5), census
    at x=3 (t=1), surface at x=4 (t=1.5), leak at x=10 (t=4.5); no draws."""
    r = O.OracleRun(_void_problem())
    tr, _ = r.run(1, seed=1, trace_cap=16)
    ev = [(int(e["type"]), e["x"], e["t"], int(e["cell"]), int(e["k"]), e["aux"]) for e in tr]
    S, SU, CE, LK = O.EV["source"], O.EV["surface"], O.EV["census"], O.EV["leak"]
    assert ev == [(S, 1.0, 0.0, -1, 0, 0.0), (SU, 2.0, 0.5, 0, 0, 1.0), (CE, 3.0, 1.0, 0, 0, 1.0),
                  (SU, 4.0, 1.5, -1, 0, 1.0), (LK, 10.0, 4.5, -1, 0, 6.0)]
    assert list(r.leak) == [0, 1, 0, 0, 0, 0]
    # track length per x-bin (1 cm each from x=1 to 10), time bins of 1 s
    mean, _ = r.mesh_stats()
    tl = mean.reshape(10, 10)
    # x in [1,3] during t in [0,1]; [3,5] during [1,2]; [5,7] in [2,3]; ...
    exp_ = np.zeros((10, 10))
    for ix in range(1, 10):
        tmid = (ix + 0.5 - 1.0) / 2.0
        exp_[int(tmid), ix] = 1.0
    assert np.array_equal(tl, exp_)


def test_hand_checked_reflection_and_diagonal():
    p = _void_problem()
    p["bc"] = np.array([1, 1, 0, 0, 0, 0], np.int32)     # reflective in x, vacuum y/z
    p["box_lo"] = np.zeros((0, 3)); p["box_hi"] = np.zeros((0, 3)); p["box_mat"] = np.zeros(0, np.int32)
    p["source"]["lo"] = p["source"]["hi"] = np.array([5.0, 5.0, 5.0])
    p["source"]["dir"] = np.array([0.6, 0.8, 0.0])
    p["speed"] = np.array([1.0])
    p["census"] = np.array([100.0])
    r = O.OracleRun(p)
    tr, _ = r.run(1, seed=1, trace_cap=16)
    # d(x=10) = 5/0.6 = 8.33 > d(y=10) = 5/0.8 = 6.25: leaks through +y at x=8.75
    assert [int(e["type"]) for e in tr] == [O.EV["source"], O.EV["leak"]]
    assert tr[1]["y"] == 10.0 and tr[1]["x"] == 5.0 + 0.6 * 6.25 and tr[1]["t"] == 6.25
    p["source"]["dir"] = np.array([0.8, 0.6, 0.0])
    r = O.OracleRun(p)
    tr, _ = r.run(1, seed=1, trace_cap=16)
    # reflects at x=10 after 6.25 (y=8.75), then leaks at y=10 after 2.0833
    assert [int(e["type"]) for e in tr] == [O.EV["source"], O.EV["surface"], O.EV["leak"]]
    assert tr[1]["x"] == 10.0 and tr[1]["ux"] == -0.8
    assert tr[2]["y"] == 10.0 and abs(tr[2]["t"] - (5 / 0.6)) < 1e-12


def _brute_force_tally(prob, trace):
    """Independent scoring: every flight segment against every space-time bin
    by clipping the segment's parameter interval to the bin box."""
    m = prob["mesh"]
    n = [int(v) for v in m["n"]]
    lo, hi = np.asarray(m["lo"], float), np.asarray(m["hi"], float)
    G = prob["sigma_t"].shape[1] if m["per_group"] else 1
    tally = np.zeros((G, n[3], n[2], n[1], n[0]))
    edges = [np.linspace(lo[a], hi[a], n[a] + 1) if np.isfinite(lo[a]) else np.array([-np.inf, np.inf])
             for a in range(4)]
    speed = np.asarray(prob["speed"], float)
    order = np.lexsort((trace["seq"], trace["tag"], trace["hist"]))
    tr = trace[order]
    for i in range(1, len(tr)):
        a, b = tr[i - 1], tr[i]
        if a["hist"] != b["hist"] or a["tag"] != b["tag"] or b["aux"] <= 0:
            continue
        d = b["aux"]
        p0 = np.array([a["x"], a["y"], a["z"]])
        u = np.array([a["ux"], a["uy"], a["uz"]])
        v = speed[a["g"]]
        gi = a["g"] if G > 1 else 0
        # per-axis parameter intervals for each bin
        iv = []
        for ax in range(3):
            e = edges[ax]
            if u[ax] == 0:
                inside = (e[:-1] <= p0[ax]) & (p0[ax] < e[1:])
                iv.append((np.where(inside, -np.inf, np.inf), np.where(inside, np.inf, -np.inf)))
            else:
                s1 = (e[:-1] - p0[ax]) / u[ax]
                s2 = (e[1:] - p0[ax]) / u[ax]
                iv.append((np.minimum(s1, s2), np.maximum(s1, s2)))
        et = edges[3]
        iv.append(((et[:-1] - a["t"]) * v, (et[1:] - a["t"]) * v))
        s_lo = np.maximum.reduce(np.meshgrid(iv[3][0], iv[2][0], iv[1][0], iv[0][0], indexing="ij"))
        s_hi = np.minimum.reduce(np.meshgrid(iv[3][1], iv[2][1], iv[1][1], iv[0][1], indexing="ij"))
        s_lo = np.maximum(s_lo, 0.0)
        s_hi = np.minimum(s_hi, d)
        tally[gi] += a["w"] * np.maximum(s_hi - s_lo, 0.0)
    return tally.ravel()


@pytest.mark.parametrize("which", ["slab", "duct"])
def test_brute_force_rescoring(which):
    if which == "slab":
        p = W.config1()
        p["mesh"]["n"] = np.array([20, 1, 1, 5], np.int32)
        nh = 400
    else:
        p = W.config2()
        p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
        p["census"] = np.array([60.0, 120.0, 200.0])
        nh = 300
    p["n_batches"] = 1
    r = O.OracleRun(p)
    tr, _ = r.run(nh, seed=23, trace_cap=100000)
    assert len(tr) < 100000
    ref = _brute_force_tally(p, tr)
    got = r.tally_sum
    scale = max(ref.max(), 1e-300)
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale * 10, np.max(np.abs(got - ref)) / scale


@pytest.mark.parametrize("cfg", ["slab", "duct", "mg"])
def test_path_conservation_and_weight_balance(cfg):
    p = {"slab": W.config1, "duct": W.config2, "mg": W.config3}[cfg]()
    N = {"slab": 20000, "duct": 3000, "mg": 1000}[cfg]
    r = O.run(p, N, seed=29)
    ws = r.wsum
    # mesh covers the geometry and [0, end time]: all track length is scored
    assert abs(r.tally_sum.sum() - ws["path"]) <= 1e-12 * ws["path"] * 10
    # analog: every source particle ends exactly once
    c = r.counters
    assert c["leak"] + c["absorb"] + c["time_end"] == c["particle"] == N
    assert ws["source"] == ws["leak"] + ws["absorb"] + ws["time_end"]


def test_implicit_capture_weight_balance():
    p = W.config2()
    p["implicit_capture"] = True
    r = O.run(p, 2000, seed=31)
    ws = r.wsum
    lhs = ws["source"] + ws["gain"] - ws["loss"]
    rhs = ws["leak"] + ws["absorb"] + ws["time_end"]
    assert abs(lhs - rhs) <= 1e-9 * ws["source"]
    assert abs(r.tally_sum.sum() - ws["path"]) <= 1e-11 * ws["path"]


def test_implicit_matches_analog_statistically():
    p = W.config1()
    ra = O.run(p, 40000, seed=37)
    pi = W.config1()
    pi["implicit_capture"] = True
    ri = O.run(pi, 40000, seed=38)
    ma, sa = ra.mesh_stats()
    mi, si = ri.mesh_stats()
    ok = (ma > 0) & (mi > 0)
    z = np.abs(ma - mi)[ok] / np.sqrt(sa[ok] ** 2 + si[ok] ** 2)
    assert np.mean(z < 3) > 0.97 and np.max(z) < 6


def test_event_cap_and_invalid():
    p = W.infinite_medium(1.0, [[0.99]], [1.0], half=5.0, t_end=1e6, nt=1)
    p["max_events"] = 5
    with pytest.raises(O.OracleError) as e:
        O.run(p, 100, seed=1)
    assert e.value.status == -4
    q = W.config1()
    q["census"] = np.array([5.0, 4.0])
    with pytest.raises(O.OracleError) as e:
        O.run(q, 1, seed=1)
    assert e.value.status == -1


def _clip_len(p, u, t0, v, d, lo, hi):
    """Length of {s in [0, d]: lo <= p + s u <= hi on each axis and
    lo_t <= t0 + s / v <= hi_t}: intersection of the slab intervals."""
    a0, a1 = 0.0, d
    for a in range(3):
        if u[a] == 0.0:
            if not (lo[a] <= p[a] <= hi[a]):
                return 0.0
            continue
        s1, s2 = (lo[a] - p[a]) / u[a], (hi[a] - p[a]) / u[a]
        a0, a1 = max(a0, min(s1, s2)), min(a1, max(s1, s2))
    a0, a1 = max(a0, (lo[3] - t0) * v), min(a1, (hi[3] - t0) * v)
    return max(a1 - a0, 0.0)


def test_score_segment_matches_clipping_per_bin():
    """Random segments (starting inside and outside the mesh in space and
    time, some axes with zero direction component) against exact clipping of
    the segment to every bin's space-time box: the walk's per-bin length
    agrees to 1e-9 (the crossing distances accumulate rounding over a few
    dozen steps), and every bin it scores is one the segment passes through."""
    rng = np.random.default_rng(20240904)
    p = W.config2()
    lo = np.array([2.0, -1.0, 0.5, 1.0])
    hi = np.array([8.0, 4.0, 6.5, 9.0])
    n = np.array([6, 5, 4, 8], np.int32)
    p["mesh"] = dict(lo=lo, hi=hi, n=n, per_group=False)
    v = 1.7
    p["speed"] = np.array([v])
    delta = (hi - lo) / n
    checked = 0
    for trial in range(200):
        x = rng.uniform(lo[:3] - 2.0, hi[:3] + 2.0)
        u = rng.normal(size=3)
        if trial % 5 == 0:
            u[trial % 3] = 0.0
            x[trial % 3] = lo[trial % 3] + delta[trial % 3] * (0.3 + (trial % 4))
        u /= np.linalg.norm(u)
        t0 = rng.uniform(0.0, 10.0)
        d = rng.uniform(0.5, 15.0)
        tally, npieces = O.score_segment(p, x, u, t0, d)
        t = tally.reshape(n[3], n[2], n[1], n[0])
        ref = np.zeros_like(t)
        for it in range(n[3]):
            for iz in range(n[2]):
                for iy in range(n[1]):
                    for ix in range(n[0]):
                        i = np.array([ix, iy, iz, it])
                        ref[it, iz, iy, ix] = _clip_len(x, u, t0, v, d, lo + i * delta, lo + (i + 1) * delta)
        np.testing.assert_allclose(t, ref, rtol=0, atol=1e-9)
        assert np.all(ref[t > 0] > 0)
        assert npieces == int(np.count_nonzero(t > 0))
        checked += int(np.count_nonzero(ref))
    assert checked > 200


def test_score_segment_hand_case():
    p = W.config2()
    p["mesh"]["n"] = np.array([60, 100, 60, 20], np.int32)
    # from (0.5,0.5,0.5) along +x for 3 cm at t=0 (v=1): bins ix 0..3 get 0.5,1,1,0.5
    tally, n = O.score_segment(p, [0.5, 0.5, 0.5], [1.0, 0.0, 0.0], 0.0, 3.0, w=2.0)
    t = tally.reshape(20, 60, 100, 60)
    assert n == 4
    assert list(t[0, 0, 0, :5]) == [1.0, 2.0, 2.0, 1.0, 0.0]
    # starting exactly on an edge moving down belongs to the lower bin
    tally, n = O.score_segment(p, [3.0, 0.5, 0.5], [-1.0, 0.0, 0.0], 0.0, 1.5)
    t = tally.reshape(20, 60, 100, 60)
    assert list(t[0, 0, 0, :4]) == [0.0, 0.5, 1.0, 0.0] and n == 2
    # crossing a time edge at t=10 splits the piece
    tally, n = O.score_segment(p, [0.2, 0.5, 0.5], [1.0, 0.0, 0.0], 9.5, 0.6)
    t = tally.reshape(20, 60, 100, 60)
    assert t[0, 0, 0, 0] == pytest.approx(0.5) and t[1, 0, 0, 0] == pytest.approx(0.1) and n == 2
