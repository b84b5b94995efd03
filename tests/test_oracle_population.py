"""Pins of the oracle's population control at census (splitting-roulette of
each intermediate census bank to a target size): every keep/kill decision
recomputed from the particle's own random stream, the deterministic
two-for-one case, the expected bank size, weight balance, and unbiased
tallies against the pulsed infinite-medium closed form and against the run
without control.  CPU only."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04668_amd import workloads as W


def _void_pulse(target, n_census=2):
    p = W._base(1)
    p["outer_lo"] = np.full(3, -50.0)
    p["outer_hi"] = np.full(3, 50.0)
    p["sigma_t"] = np.array([[0.0]])
    p["sigma_s"] = np.array([[[0.0]]])
    p["mesh"] = dict(lo=np.array([-50.0, -50.0, -50.0, 0.0]), hi=np.array([50.0, 50.0, 50.0, 10.0]),
                     n=np.array([2, 1, 1, 5], np.int32), per_group=False)
    p["census"] = np.linspace(0.0, 10.0, n_census + 1)[1:]
    p["n_batches"] = 1
    p["population_control"] = dict(target=target)
    return p


def test_two_for_one_is_deterministic():
    """Every particle reaches the census at t = 5 with weight 1; target 2 per
    history gives w_T = 1/2 and n = floor(2 + xi) = 2 copies of weight 1/2."""
    p = _void_pulse(2.0)
    n = 500
    r = O.OracleRun(p)
    tr, _ = r.run(n, seed=3, trace_cap=100000)
    keep = tr[tr["type"] == O.EV["pc_keep"]]
    assert len(keep) == n and np.all(keep["aux"] == 2.0) and np.all(keep["w"] == 0.5)
    c = r.counters
    assert c["pc_copy"] == n and c["pc_kill"] == 0 and c["particle"] == 2 * n
    assert c["time_end"] == 2 * n
    assert r.wsum["time_end"] == float(n) and r.wsum["gain"] == 0.0 and r.wsum["loss"] == 0.0


def test_roulette_decisions_follow_each_particles_stream():
    """Target 0.3 per history: w_T = 1/0.3, each unit-weight particle survives
    iff xi * w_T < 1, xi being the next draw of its own stream (the census
    record carries the stream position)."""
    p = _void_pulse(0.3)
    n = 2000
    seed = 7
    r = O.OracleRun(p)
    tr, _ = r.run(n, seed=seed, trace_cap=100000)
    cen = tr[tr["type"] == O.EV["census"]]
    assert len(cen) == n
    M = math.floor(0.3 * n + 0.5)
    wq = n * 2 ** 32                              # floor(1 * 2^32) per particle
    wt = (wq * 2.0 ** -32) / M
    dec = {}
    for e in tr[(tr["type"] == O.EV["pc_keep"]) | (tr["type"] == O.EV["pc_kill"])]:
        dec[(int(e["hist"]), int(e["tag"]))] = int(e["type"])
    assert len(dec) == n
    survivors = 0
    for e in cen:
        xi = O.uniform(seed, int(e["hist"]), 0, int(e["tag"]), int(e["k"]))
        keep = xi * wt < 1.0
        survivors += keep
        assert dec[(int(e["hist"]), int(e["tag"]))] == (O.EV["pc_keep"] if keep else O.EV["pc_kill"])
    assert survivors == r.counters["time_end"]
    assert abs(survivors - M) < 4 * math.sqrt(M)


def test_bank_size_tracks_target_and_weight_balances():
    p = W.infinite_medium(1.0, [[0.9]], [1.0], half=5.0, t_end=8.0, nt=8)
    p["census"] = np.linspace(1.0, 8.0, 8)
    p["population_control"] = dict(target=1.5)
    p["n_batches"] = 4
    n = 4000
    r = O.OracleRun(p)
    tr, _ = r.run(n, seed=11, trace_cap=400000)
    keep = tr[tr["type"] == O.EV["pc_keep"]]
    # per census time the kept population sums to about 1.5 per history
    for tc in p["census"][:-1]:
        sel = keep[keep["t"] == tc]
        tot = sel["aux"].sum()
        M = 1.5 * n / 4                          # per batch, four batches
        assert abs(tot - 4 * M) < 5 * math.sqrt(4 * M), (tc, tot)
    ws = r.wsum
    lhs = ws["source"] + ws["gain"] - ws["loss"]
    rhs = ws["leak"] + ws["absorb"] + ws["time_end"]
    assert abs(lhs - rhs) <= 1e-9 * ws["source"]


@pytest.mark.parametrize("target", [0.4, 3.0])
def test_population_control_unbiased_pulsed_infinite_medium(target):
    sig_t, sig_s, v = 1.0, 0.7, 1.0
    sig_a = sig_t - sig_s
    p = W.infinite_medium(sig_t, [[sig_s]], [v], half=5.0, t_end=6.0, nt=6)
    p["census"] = np.linspace(1.0, 6.0, 6)
    p["population_control"] = dict(target=target)
    N = 30000
    r = O.run(p, N, seed=17)
    mean, se = r.mesh_stats()
    edges = np.linspace(0, 6.0, 7)
    exp_ = (np.exp(-v * sig_a * edges[:-1]) - np.exp(-v * sig_a * edges[1:])) / sig_a
    assert np.all(np.abs(mean - exp_) < 4 * se), (mean, exp_, se)
    assert r.counters["pc_kill"] + r.counters["pc_copy"] > 1000


def test_population_control_matches_uncontrolled_duct():
    p = W.config2(n_census=4)
    p["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    N = 20000
    ra = O.run(p, N, seed=21)
    q = W.config2(n_census=4)
    q["mesh"]["n"] = np.array([6, 10, 6, 4], np.int32)
    q["population_control"] = dict(target=0.5)
    rp = O.run(q, N, seed=22)
    ma, sa = ra.mesh_stats()
    mp, sp = rp.mesh_stats()
    ok = (sa > 0) & (sp > 0)
    z = np.abs(ma - mp)[ok] / np.sqrt(sa[ok] ** 2 + sp[ok] ** 2)
    assert np.mean(z < 3) > 0.95 and np.max(z) < 5
    da, dsa = ra.detector_stats()
    dp, dsp = rp.detector_stats()
    assert abs(da - dp) < 4 * math.hypot(dsa, dsp)
