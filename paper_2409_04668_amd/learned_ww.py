"""Learned weight windows: importance estimate -> GPU MLP training -> windows.

Pipeline (every numerical step runs in libmcdc's kernels; this module only
orchestrates calls and assembles the training set):
  1. analog runs with the coarse importance estimate on (forward estimate:
     each flight start in a coarse space-time-group cell adds the detector score
     that its history still makes afterwards, and one unit of weight);
  2. training set: one point per cell, input = cell centre scaled to [-1,1]
     over the outer box and [0, end time] plus a group one-hot, target =
     log(score / weight); cells that were visited but never led to a score get
     a floor target one decade below the smallest positive estimate;
  3. full-batch Adam on the GPU (mcdc_mlp_train) for the log-importance MLP
     in -> 64 -> 64 -> 1;
  4. log K = log of the mean importance over source samples, so that source
     particles (weight 1) start near their target weight;
  5. mcdc_set_ww_mlp turns splitting/roulette on.
The analog run stays the reference: weight windows change variance, not the
expected tallies.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import mcdc
from . import workloads as W


def _cell_centres(prob: dict, n4, G: int):
    nx, ny, nz, nt = [int(v) for v in n4]
    g, it, iz, iy, ix = np.meshgrid(np.arange(G), np.arange(nt), np.arange(nz), np.arange(ny),
                                    np.arange(nx), indexing="ij")
    cx = (ix.ravel() + 0.5) / nx
    cy = (iy.ravel() + 0.5) / ny
    cz = (iz.ravel() + 0.5) / nz
    ct = (it.ravel() + 0.5) / nt
    X = np.zeros((cx.size, 4 + G), np.float32)
    X[:, 0] = 2 * cx - 1
    X[:, 1] = 2 * cy - 1
    X[:, 2] = 2 * cz - 1
    X[:, 3] = 2 * ct - 1
    X[np.arange(cx.size), 4 + g.ravel()] = 1.0
    return X


def importance_estimate(prob: dict, n_runs: int, n_per_run: int, seed0: int, grid=None,
                        options=None):
    """Run analog histories with the coarse importance estimate on; returns
    (score, weight, seconds)."""
    import torch
    q = W.with_(prob, importance=grid or W.coarse_importance_grid(), ww=None,
                implicit_capture=False)
    gp = mcdc.Problem(q, options)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_runs):
        gp.run(n_per_run, seed0 + i)
    S, Wt = gp.importance()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gp.close()
    return S, Wt, dt, q["importance"]["n"]


def training_set(prob: dict, S, Wt, n4):
    G = prob["sigma_t"].shape[1]
    X = _cell_centres(prob, n4, G)
    pos = (S > 0) & (Wt > 0)
    if not pos.any():
        raise RuntimeError("importance estimate has no scoring cell: run more histories")
    I = np.zeros_like(S)
    I[pos] = S[pos] / Wt[pos]
    floor = I[pos].min() / 10.0
    visited = Wt > 0
    y = np.where(pos, np.log(np.where(pos, I, 1.0)), np.log(floor)).astype(np.float32)
    wt = np.where(pos, np.sqrt(Wt), 0.25 * np.sqrt(Wt)).astype(np.float32)
    sel = visited
    return X[sel], y[sel], wt[sel]


def _init_params(in_dim: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    H = mcdc.HIDDEN
    W1 = rng.uniform(-1, 1, (H, in_dim)) * np.sqrt(6.0 / in_dim)
    W2 = rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H)
    W3 = rng.uniform(-1, 1, (H,)) * np.sqrt(6.0 / H)
    return np.concatenate([W1.ravel(), np.full(H, 0.01), W2.ravel(), np.full(H, 0.01), W3,
                           np.zeros(1)]).astype(np.float32)


def gpu_train(X, y, wt, steps=3000, lr=3e-3, seed=1, params=None, device="cuda:0"):
    """Train the log-importance MLP with the library's kernels (full batch,
    Adam).  Returns (params, loss history, seconds)."""
    import torch
    n, in_dim = X.shape
    p0 = _init_params(in_dim, seed) if params is None else np.asarray(params, np.float32)
    dev = torch.device(device)
    tX = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(dev)
    ty = torch.from_numpy(np.ascontiguousarray(y, np.float32)).to(dev)
    tw = torch.from_numpy(np.ascontiguousarray(wt, np.float32)).to(dev)
    tp = torch.from_numpy(p0.copy()).to(dev)
    tm = torch.zeros_like(tp)
    tv = torch.zeros_like(tp)
    tg = torch.zeros_like(tp)
    tl = torch.zeros(max(steps, 1), dtype=torch.float32, device=dev)
    scratch = torch.empty(int(mcdc._lib.mcdc_mlp_scratch_bytes(in_dim, n)), dtype=torch.uint8,
                          device=dev)
    o = mcdc.TrainOpts()
    o.steps, o.lr, o.beta1, o.beta2, o.eps = steps, lr, 0.9, 0.999, 1e-8
    step = C.c_int32(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mcdc.check(mcdc._lib.mcdc_mlp_train(mcdc._ptr(tp), in_dim, mcdc._ptr(tX), mcdc._ptr(ty),
                                        mcdc._ptr(tw), n, mcdc._ptr(tm), mcdc._ptr(tv),
                                        mcdc._ptr(tg), C.byref(o), C.byref(step), mcdc._ptr(tl),
                                        mcdc._ptr(scratch), mcdc._stream_ptr()), "mlp_train")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return tp.cpu().numpy(), tl.cpu().numpy(), dt


def gpu_forward(params, X, device="cuda:0"):
    import torch
    dev = torch.device(device)
    tX = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(dev)
    tp = torch.from_numpy(np.ascontiguousarray(params, np.float32)).to(dev)
    out = torch.empty(X.shape[0], dtype=torch.float32, device=dev)
    mcdc.check(mcdc._lib.mcdc_mlp_forward(mcdc._ptr(tp), X.shape[1], mcdc._ptr(tX), X.shape[0],
                                          mcdc._ptr(out), mcdc._stream_ptr()), "mlp_forward")
    return out.cpu().numpy()


def source_log_k(prob: dict, params, n=10000, seed=3):
    """log of the mean importance exp(y) over source samples."""
    rng = np.random.default_rng(seed)
    src = prob["source"]
    lo = np.asarray(prob["outer_lo"], float)
    hi = np.asarray(prob["outer_hi"], float)
    t_end = float(prob["census"][-1])
    G = prob["sigma_t"].shape[1]
    if src["kind"] == "box":
        pos = rng.uniform(np.asarray(src["lo"]), np.asarray(src["hi"]), size=(n, 3))
    else:
        pos = np.tile(np.asarray(src["lo"], float), (n, 1))
    t = rng.uniform(src["t0"], src["t1"], n) if src["t1"] > src["t0"] else np.full(n, src["t0"])
    X = np.zeros((n, 4 + G), np.float32)
    X[:, :3] = 2 * (pos - lo) / (hi - lo) - 1
    X[:, 3] = 2 * t / t_end - 1
    X[:, 4 + int(src["group"])] = 1.0
    yv = gpu_forward(params, X).astype(np.float64)
    m = yv.max()
    return float(m + np.log(np.mean(np.exp(yv - m))))


def build_ww(prob: dict, n_runs=20, n_per_run=1_000_000, seed0=W.ROOT_SEED + 1, steps=3000,
             lr=3e-3, ratio=5.0, n_max=10):
    """Whole pipeline; returns (ww dict for the problem, info dict)."""
    S, Wt, t_imp, n4 = importance_estimate(prob, n_runs, n_per_run, seed0)
    X, y, wt = training_set(prob, S, Wt, n4)
    params, losses, t_train = gpu_train(X, y, wt, steps=steps, lr=lr)
    logk = source_log_k(prob, params)
    ww = dict(params=params, hidden=mcdc.HIDDEN, logk=logk, ratio=ratio, n_max=n_max)
    info = dict(importance_seconds=t_imp, train_seconds=t_train, n_points=int(X.shape[0]),
                n_scoring_cells=int((S > 0).sum()), loss_first=float(losses[0]),
                loss_last=float(losses[-1]), logk=logk)
    return ww, info


def fom_run(prob: dict, n_hist: int, seed: int, options=None, chunk: int = 50_000_000):
    """Run n_hist histories; returns (detector mean, relative error, GPU seconds)."""
    import torch
    gp = mcdc.Problem(prob, options)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    i = 0
    while done < n_hist:
        n = min(chunk, n_hist - done)
        gp.run(n, seed + i)
        done += n
        i += 1
    m, r = gp.tallies(mcdc.TALLY_DETECTOR)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    c = gp.counters()
    gp.close()
    return float(m[0]), float(r[0]), dt, c


def fom_at_target(prob: dict, seed: int, target=0.01, pilot=2_000_000, options=None,
                  max_hist=4_000_000_000):
    """Pilot run -> N such that the detector relative error reaches `target`
    -> run at that N.  Returns a dict with N, mean, rel_err, seconds, FOM."""
    m, r, dt, _ = fom_run(prob, pilot, seed, options)
    if not (r > 0):
        raise RuntimeError("pilot run scored nothing on the detector")
    n = int(min(max_hist, max(pilot, np.ceil(pilot * (r / target) ** 2 * 1.02))))
    m, r, dt, c = fom_run(prob, n, seed + 1000, options)
    return dict(n=n, mean=m, rel_err=r, seconds=dt, fom=1.0 / (r * r * dt),
                histories_per_s=n / dt, splits=c["splits"], rr_kills=c["rr_kills"],
                particles=c["particles"])
