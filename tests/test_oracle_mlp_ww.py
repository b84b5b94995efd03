"""Pins of the oracle's learned-importance parts: the FP64 MLP reference against
torch autograd and finite differences, the FP32 inference used inside the
transport loop against the FP64 forward, Adam against torch.optim.Adam,
weight-window unbiasedness and bookkeeping, and the forward importance
estimate on a hand-checked void problem.  CPU only."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp as M
from oracle import oracle as O
from paper_2409_04668_amd import workloads as W

IN, H = 5, 64


def _torch_net(params):
    W1, b1, W2, b2, W3, b3 = [torch.tensor(a, dtype=torch.float64) for a in M.unpack(params, IN, H)]
    net = torch.nn.Sequential(torch.nn.Linear(IN, H), torch.nn.ReLU(), torch.nn.Linear(H, H),
                              torch.nn.ReLU(), torch.nn.Linear(H, 1)).double()
    with torch.no_grad():
        net[0].weight.copy_(W1); net[0].bias.copy_(b1)
        net[2].weight.copy_(W2); net[2].bias.copy_(b2)
        net[4].weight.copy_(W3.reshape(1, H)); net[4].bias.copy_(b3)
    return net


def _data(n=300, seed=3):
    rng = np.random.default_rng(seed)
    X = np.concatenate([rng.uniform(-1, 1, (n, 4)), np.ones((n, 1))], axis=1)
    y = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2] - 0.5 * X[:, 3]
    wt = rng.uniform(0.5, 2.0, n)
    return X, y, wt


def _torch_flat_grad(net):
    g = [net[0].weight.grad, net[0].bias.grad, net[2].weight.grad, net[2].bias.grad,
         net[4].weight.grad.reshape(-1), net[4].bias.grad]
    return torch.cat([t.reshape(-1) for t in g]).numpy()


def test_forward_and_grad_match_torch_autograd():
    p = M.init_params(IN, H, seed=1).astype(np.float64)
    p[H * IN:H * IN + H] = np.random.default_rng(2).normal(0, 0.1, H)      # nonzero b1
    X, y, wt = _data()
    net = _torch_net(p)
    out_t = net(torch.tensor(X)).reshape(-1)
    out_n, _ = M.forward(p, X, IN, H)
    assert np.max(np.abs(out_t.detach().numpy() - out_n)) < 1e-12
    wt_t = torch.tensor(wt)
    L = torch.sum(wt_t * (out_t - torch.tensor(y)) ** 2) / wt_t.sum()
    L.backward()
    g_t = _torch_flat_grad(net)
    g_n = M.grad(p, X, y, wt, IN, H)
    assert abs(L.item() - M.loss(p, X, y, wt, IN, H)) < 1e-12
    assert np.max(np.abs(g_t - g_n)) <= 1e-10 * np.max(np.abs(g_t))


def test_grad_matches_finite_differences():
    p = M.init_params(IN, H, seed=4).astype(np.float64)
    X, y, wt = _data(60, seed=5)
    g = M.grad(p, X, y, wt, IN, H)
    rng = np.random.default_rng(6)
    h = 1e-6
    idx = rng.choice(p.size, 80, replace=False)
    _, (_, z1, _, z2, _) = M.forward(p, X, IN, H)
    checked = 0
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        # skip parameters whose perturbation moves a pre-activation across 0
        _, (_, z1p, _, z2p, _) = M.forward(pp, X, IN, H)
        _, (_, z1m, _, z2m, _) = M.forward(pm, X, IN, H)
        if np.any(np.sign(z1p) != np.sign(z1m)) or np.any(np.sign(z2p) != np.sign(z2m)):
            continue
        fd = (M.loss(pp, X, y, wt, IN, H) - M.loss(pm, X, y, wt, IN, H)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])
        checked += 1
    assert checked > 40


def test_fp32_inference_matches_fp64_forward():
    p = M.init_params(IN, H, seed=7)
    X, _, _ = _data(200, seed=8)
    ref, _ = M.forward(p.astype(np.float64), X.astype(np.float32).astype(np.float64), IN, H)
    got = np.array([O.mlp_f32(p, IN, H, x) for x in X])
    scale = np.max(np.abs(ref)) + 1.0
    assert np.max(np.abs(got - ref)) < 2e-5 * scale


def test_adam_matches_torch():
    p0 = M.init_params(IN, H, seed=9).astype(np.float64)
    X, y, wt = _data(100, seed=10)
    net = _torch_net(p0)
    opt = torch.optim.Adam(net.parameters(), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    Xt, yt, wtt = torch.tensor(X), torch.tensor(y), torch.tensor(wt)
    for step in range(1, 6):
        opt.zero_grad()
        out = net(Xt).reshape(-1)
        L = torch.sum(wtt * (out - yt) ** 2) / wtt.sum()
        L.backward()
        opt.step()
        p, m, v = M.adam_step(p, M.grad(p, X, y, wt, IN, H), m, v, step, 1e-3)
    tp = np.concatenate([t.detach().reshape(-1).numpy() for t in net.parameters()])
    assert np.max(np.abs(tp - p)) < 1e-12


def test_adam_decreases_loss():
    p = M.init_params(IN, H, seed=11).astype(np.float64)
    X, y, wt = _data(200, seed=12)
    m, v = np.zeros_like(p), np.zeros_like(p)
    losses = []
    for step in range(1, 51):
        losses.append(M.loss(p, X, y, wt, IN, H))
        p, m, v = M.adam_step(p, M.grad(p, X, y, wt, IN, H), m, v, step, 1e-3)
    assert losses[-1] < 0.7 * losses[0]
    assert all(b <= a * 1.001 for a, b in zip(losses, losses[1:]))


# ---------------------------------------------------------------------------
# weight windows
# ---------------------------------------------------------------------------

def _box_problem():
    p = W._base(1)
    p["outer_lo"] = np.zeros(3)
    p["outer_hi"] = np.full(3, 20.0)
    p["sigma_t"] = np.array([[0.5]])
    p["sigma_s"] = np.array([[[0.4]]])
    p["speed"] = np.array([1.0])
    p["source"] = dict(kind="point", lo=np.full(3, 10.0), hi=np.full(3, 10.0), t0=0.0, t1=0.0,
                       isotropic=True, dir=np.array([1.0, 0.0, 0.0]), group=0)
    p["mesh"] = dict(lo=np.array([0.0, 0.0, 0.0, 0.0]), hi=np.array([20.0, 20.0, 20.0, 40.0]),
                     n=np.array([10, 2, 2, 4], np.int32), per_group=False)
    p["census"] = np.array([40.0])
    p["detector"] = dict(lo=np.array([16.0, 0.0, 0.0]), hi=np.array([20.0, 20.0, 20.0]))
    return p


def _ramp_mlp(slope):
    """y = slope * xhat_x exactly (in FP32): one ReLU path carries xhat_x + 1."""
    prm = np.zeros(M.n_params(IN, H), np.float32)
    o = 0
    prm[o + 0] = 1.0                       # W1[0][0]
    o += H * IN
    prm[o + 0] = 1.0                       # b1[0]
    o += H
    prm[o + 0] = 1.0                       # W2[0][0]
    o += H * H + H
    prm[o + 0] = slope                     # W3[0]
    o += H
    prm[o] = -slope                        # b3
    return prm


def test_constant_importance_is_bit_identical_to_analog():
    p = _box_problem()
    ra = O.OracleRun(p)
    ta, xa = ra.run(3000, seed=41, trace_cap=200000, per_history=True)
    q = _box_problem()
    q["ww"] = dict(params=np.zeros(M.n_params(IN, H), np.float32), hidden=H, logk=0.0,
                   ratio=5.0, n_max=10)
    rw = O.OracleRun(q)
    tw, xw = rw.run(3000, seed=41, trace_cap=200000, per_history=True)
    assert np.array_equal(ta, tw)
    assert np.array_equal(xa, xw)
    assert np.array_equal(ra.tally_sum, rw.tally_sum)


def test_weight_windows_unbiased_and_balanced():
    p = _box_problem()
    N = 20000
    ra = O.run(p, N, seed=43)
    q = _box_problem()
    q["ww"] = dict(params=_ramp_mlp(2.0), hidden=H, logk=0.0, ratio=5.0, n_max=10)
    rw = O.run(q, N, seed=44)
    c = rw.counters
    assert c["split"] > 1000 and c["rr_kill"] > 1000
    ws = rw.wsum
    lhs = ws["source"] + ws["gain"] - ws["loss"]
    rhs = ws["leak"] + ws["absorb"] + ws["time_end"]
    assert abs(lhs - rhs) <= 1e-9 * ws["source"]
    assert abs(rw.tally_sum.sum() - ws["path"]) <= 1e-11 * ws["path"]
    ma, sa = ra.mesh_stats()
    mw, sw = rw.mesh_stats()
    ok = (ma > 0) & (mw > 0)
    z = np.abs(ma - mw)[ok] / np.sqrt(sa[ok] ** 2 + sw[ok] ** 2)
    assert np.mean(z < 3) > 0.95 and np.max(z) < 5
    da, dsa = ra.detector_stats()
    dw, dsw = rw.detector_stats()
    assert abs(da - dw) < 3.5 * math.hypot(dsa, dsw)
    # splitting toward the detector lowers its relative error per history
    assert dsw / dw < dsa / da


def test_split_expected_weight_unit():
    """One collision-free check: a particle far above its window splits into
    n = min(ceil(w/w_T), n_max) copies of weight w/n (total weight kept)."""
    p = _box_problem()
    p["sigma_t"] = np.array([[0.0]])
    p["sigma_s"] = np.array([[[0.0]]])
    p["source"]["isotropic"] = False
    p["box_lo"] = np.array([[11.0, 0.0, 0.0]])
    p["box_hi"] = np.array([[12.0, 20.0, 20.0]])
    p["box_mat"] = np.array([0], np.int32)
    # at the crossing xhat = 0.1: w_T = exp(-0.6) ~ 0.55 < w_U(1) -> two copies of 0.5
    p["ww"] = dict(params=_ramp_mlp(6.0), hidden=H, logk=0.0, ratio=5.0, n_max=10)
    r = O.OracleRun(p)
    tr, _ = r.run(1, seed=1, trace_cap=100)
    sp = tr[tr["type"] == O.EV["split"]]
    assert len(sp) >= 1
    first = sp[0]
    assert first["x"] == 11.0
    n = int(first["aux"])
    assert n == 2 and first["w"] == 0.5
    wt = math.exp(-6.0 * 0.1)
    assert math.ceil(1.0 / wt) == n
    # every particle's weight ends up leaking through +x
    assert abs(r.leak[1] - 1.0) < 1e-15 and r.counters["particle"] == 2


def test_importance_estimate_hand_case():
    p = W._base(1)
    p["outer_lo"] = np.zeros(3)
    p["outer_hi"] = np.full(3, 10.0)
    p["box_lo"] = np.array([[2.0, 0.0, 0.0], [7.0, 0.0, 0.0]])
    p["box_hi"] = np.array([[4.0, 10.0, 10.0], [9.0, 10.0, 10.0]])
    p["box_mat"] = np.array([0, 0], np.int32)
    p["sigma_t"] = np.zeros((1, 1))
    p["sigma_s"] = np.zeros((1, 1, 1))
    p["source"] = dict(kind="point", lo=np.array([1.0, 5.0, 5.0]), hi=np.array([1.0, 5.0, 5.0]),
                       t0=0.0, t1=0.0, isotropic=False, dir=np.array([1.0, 0.0, 0.0]), group=0)
    p["mesh"] = dict(lo=np.array([0.0, 0.0, 0.0, 0.0]), hi=np.array([10.0, 10.0, 10.0, 100.0]),
                     n=np.array([1, 1, 1, 1], np.int32), per_group=False)
    p["census"] = np.array([100.0])
    p["detector"] = dict(lo=np.array([6.0, 0.0, 0.0]), hi=np.array([8.0, 10.0, 10.0]))
    p["importance"] = dict(n=np.array([2, 1, 1, 1], np.int32))
    r = O.run(p, 3, seed=1)
    # flight starts x=1,2,4 (cell 0, score so far 0) and x=7,9 (cell 1, 1 and 2); final 2
    assert list(r.imp_weight) == [9.0, 6.0]
    assert list(r.imp_score) == [18.0, 3.0]


def test_output_clamp_to_a_point_is_constant_importance():
    """Clamping the network output to [0, 0] makes w_T = 1 everywhere, so an
    analog run (weights stay 1, inside [1/3, 5/3]) is untouched bit for bit."""
    p = _box_problem()
    ra = O.OracleRun(p)
    ta, _ = ra.run(2000, seed=47, trace_cap=200000)
    q = _box_problem()
    q["ww"] = dict(params=_ramp_mlp(5.0), hidden=H, logk=0.0, ratio=5.0, n_max=10,
                   ymin=0.0, ymax=0.0)
    rq = O.OracleRun(q)
    tq, _ = rq.run(2000, seed=47, trace_cap=200000)
    assert np.array_equal(ta, tq)
    q["ww"]["ymax"] = 5.0                 # unclamped above: splits happen
    rs = O.run(q, 2000, seed=47)
    assert rs.counters["split"] > 0


# ---------------------------------------------------------------------------
# weight-window map (network evaluated once per map cell centre)
# ---------------------------------------------------------------------------

def test_ww_map_is_network_at_cell_centres():
    p = _box_problem()
    prm = M.init_params(IN, H, seed=5)
    dims = (3, 4, 5, 2)
    # clamp range inside the network's output range so some cells are clamped
    p["ww"] = dict(params=prm, hidden=H, logk=0.3, ratio=5.0, n_max=10, ymin=-0.5, ymax=0.5,
                   map=dims)
    got = O.ww_map(p)
    assert got.shape == (1, dims[3], dims[2], dims[1], dims[0])
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in dims], indexing="ij"), -1).reshape(-1, 4)
    X = np.zeros((len(idx), IN))
    X[:, :4] = (2.0 * ((idx + 0.5) / np.array(dims)) - 1.0).astype(np.float32)
    X[:, 4] = 1.0
    y = np.clip(M.forward(prm, X, IN, H)[0], -0.5, 0.5)
    want = np.exp(0.3 - y)
    clamped = (y == -0.5) | (y == 0.5)
    assert clamped.any() and (~clamped).any()
    g = got[0].transpose(3, 2, 1, 0).reshape(-1)          # -> [ix][iy][iz][it]
    assert np.allclose(g, want, rtol=2e-6, atol=0)


def test_ww_map_cell_matches_floor_rule():
    p = _box_problem()
    dims = (7, 3, 5, 4)
    p["ww"] = dict(params=np.zeros(M.n_params(IN, H), np.float32), hidden=H, logk=0.0,
                   map=dims)
    rng = np.random.default_rng(11)
    pts = rng.uniform(-2.0, 22.0, (400, 3))
    pts[:5] = [[0.0, 0.0, 0.0], [20.0, 20.0, 20.0], [10.0, 10.0, 10.0],
               [20.0 / 7.0 * 3.0, 1e-300, 19.999999], [-1e-12, 20.0 + 1e-12, 4.0]]
    ts = rng.uniform(-1.0, 41.0, 400)
    ts[:3] = [0.0, 40.0, 10.0]
    for pt, t in zip(pts, ts):
        want = 0
        for a in (3, 2, 1, 0):
            v = t if a == 3 else pt[a]
            span = 40.0 if a == 3 else 20.0
            i = math.floor(v / span * dims[a])
            i = min(max(i, 0), dims[a] - 1)
            want = want * dims[a] + i
        got = O.ww_map_cell(p, pt, t)
        # the oracle scales by 1/span: allow a one-cell difference only on exact cell faces
        if got != want:
            f = [(t if a == 3 else pt[a]) / (40.0 if a == 3 else 20.0) * dims[a] for a in range(4)]
            assert any(abs(x - round(x)) < 1e-12 for x in f), (pt, t, got, want)


def test_ww_map_split_hand_case():
    """Void problem with one interior box (faces x=11, x=12), ramp network
    y = 6 xhat, map 10 cells along x.  At x=11 the map cell is 5 (centre
    xhat = 0.1): w_T = exp(-0.6), so weight 1 splits in two; at x=12 the cell
    is 6 (centre xhat = 0.3): w_T = exp(-1.8) ~ 0.165, window [0.055, 0.275],
    so each half splits into ceil(0.5 / 0.165) = 4 copies of 0.125.  The
    network at the crossing point itself (xhat = 0.2) would give no split."""
    p = _box_problem()
    p["sigma_t"] = np.array([[0.0]])
    p["sigma_s"] = np.array([[[0.0]]])
    p["source"]["isotropic"] = False
    p["box_lo"] = np.array([[11.0, 0.0, 0.0]])
    p["box_hi"] = np.array([[12.0, 20.0, 20.0]])
    p["box_mat"] = np.array([0], np.int32)
    p["ww"] = dict(params=_ramp_mlp(6.0), hidden=H, logk=0.0, ratio=5.0, n_max=10,
                   map=(10, 1, 1, 1))
    r = O.OracleRun(p)
    tr, _ = r.run(1, seed=1, trace_cap=100)
    sp = tr[tr["type"] == O.EV["split"]]
    assert [int(s["aux"]) for s in sp] == [2, 4, 4]
    assert [float(s["x"]) for s in sp] == [11.0, 12.0, 12.0]
    assert [float(s["w"]) for s in sp] == [0.5, 0.125, 0.125]
    assert math.ceil(0.5 / math.exp(-1.8)) == 4
    assert abs(r.leak[1] - 1.0) < 1e-15 and r.counters["particle"] == 8


def test_ww_map_unbiased():
    p = _box_problem()
    N = 20000
    ra = O.run(p, N, seed=43)
    q = _box_problem()
    q["ww"] = dict(params=_ramp_mlp(2.0), hidden=H, logk=0.0, ratio=5.0, n_max=10,
                   map=(10, 4, 4, 8))
    rw = O.run(q, N, seed=44)
    c = rw.counters
    assert c["split"] > 1000 and c["rr_kill"] > 1000
    ws = rw.wsum
    lhs = ws["source"] + ws["gain"] - ws["loss"]
    rhs = ws["leak"] + ws["absorb"] + ws["time_end"]
    assert abs(lhs - rhs) <= 1e-9 * ws["source"]
    ma, sa = ra.mesh_stats()
    mw, sw = rw.mesh_stats()
    ok = (ma > 0) & (mw > 0)
    z = np.abs(ma - mw)[ok] / np.sqrt(sa[ok] ** 2 + sw[ok] ** 2)
    assert np.mean(z < 3) > 0.95 and np.max(z) < 5
    da, dsa = ra.detector_stats()
    dw, dsw = rw.detector_stats()
    assert abs(da - dw) < 3.5 * math.hypot(dsa, dsw)
    assert dsw / dw < dsa / da


def test_ww_map_invalid_dims_rejected():
    q = _box_problem()
    q["ww"] = dict(params=np.zeros(M.n_params(IN, H), np.float32), hidden=H, logk=0.0,
                   map=(4, 0, 4, 4))
    with pytest.raises(Exception):
        O.run(q, 10, seed=1)
