"""Learned weight windows: importance tallies -> GPU MLP training -> windows.

Every numerical step runs in libmcdc's kernels; this module orchestrates the
calls and assembles the training set.

Importance data (tallies the transport itself produces), one of:
  * reciprocal runs (one energy group): for one-group transport with isotropic
    scattering, the expected detector track length of a particle emitted
    isotropically at x equals the detector volume times the scalar flux at x
    from a uniform isotropic source in the detector (reciprocity), and
    transport is invariant under time shifts, so the importance of (x, t) is
    the flux at x from a detector source at time 0 accumulated over the
    remaining horizon T_end - t.  The runs use the same problem with the
    source moved into the detector and a coarse space-time tally; the
    horizon sum is a cumulative sum over time bins.
  * forward estimate (any number of groups): analog runs with the coarse
    importance estimate on (each flight start in a coarse cell adds the
    detector score its history still makes afterwards); sparse when the
    detector is rarely reached.
Then: the training set is one point per coarse cell with a positive estimate
(input = cell centre scaled to [-1,1] over the outer box and [0, T_end] plus a
group one-hot; target = log importance); full-batch Adam on the GPU
(mcdc_mlp_train); log K = log of the mean importance over source samples so
that source particles start inside their windows; and the network output is
clamped at run time to the range of its training targets.  The transport then
evaluates the network at every check, or (``map_dims``) reads w_T from the
network baked once onto a regular cell-centre map (mcdc_set_ww_map).

Weight windows change the variance, not the expected tallies; the analog run
stays the reference for both the tallies and the figure of merit.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import mcdc
from . import workloads as W


def _cell_inputs(n4, G: int):
    """Inputs of the cell centres in tally order [g][t][z][y][x]."""
    nx, ny, nz, nt = [int(v) for v in n4]
    g, it, iz, iy, ix = np.meshgrid(np.arange(G), np.arange(nt), np.arange(nz), np.arange(ny),
                                    np.arange(nx), indexing="ij")
    X = np.zeros((ix.size, 4 + G), np.float32)
    X[:, 0] = 2 * (ix.ravel() + 0.5) / nx - 1
    X[:, 1] = 2 * (iy.ravel() + 0.5) / ny - 1
    X[:, 2] = 2 * (iz.ravel() + 0.5) / nz - 1
    X[:, 3] = 2 * (it.ravel() + 0.5) / nt - 1
    X[np.arange(ix.size), 4 + g.ravel()] = 1.0
    return X


def reciprocal_importance(prob: dict, n_runs=20, n_per_run=1_000_000, seed0=W.ROOT_SEED + 1,
                          grid=None, options=None):
    """Importance I[t][z][y][x] on the coarse grid from runs with the source in
    the detector (one group only).  Returns (I, seconds, grid cells n4)."""
    import torch
    if prob["sigma_t"].shape[1] != 1:
        raise ValueError("reciprocal importance needs one energy group")
    det = prob["detector"]
    if det is None:
        raise ValueError("the problem has no detector")
    n4 = np.asarray((grid or W.coarse_importance_grid())["n"], np.int32)
    t_end = float(prob["census"][-1])
    q = W.with_(prob, ww=None, importance=None, detector=None, n_batches=1)
    q["source"] = dict(kind="box", lo=np.asarray(det["lo"], float), hi=np.asarray(det["hi"], float),
                       t0=0.0, t1=0.0, isotropic=True, dir=np.array([1.0, 0.0, 0.0]), group=0)
    lo = np.asarray(prob["outer_lo"], float)
    hi = np.asarray(prob["outer_hi"], float)
    q["mesh"] = dict(lo=np.array([lo[0], lo[1], lo[2], 0.0]), hi=np.array([hi[0], hi[1], hi[2], t_end]),
                     n=n4, per_group=False)
    gp = mcdc.Problem(q, options)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_runs):
        gp.run(n_per_run, seed0 + i)
    s, _ = gp.raw()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gp.close()
    nx, ny, nz, nt = [int(v) for v in n4]
    vol = np.prod((hi - lo) / n4[:3])
    T = s.reshape(nt, nz, ny, nx) / (n_runs * n_per_run) / vol      # flux-time per bin
    cum = np.cumsum(T, axis=0)
    dtb = t_end / nt
    I = np.zeros_like(T)
    for b in range(nt):
        horizon = t_end - (b + 0.5) * dtb
        full = int(horizon // dtb)
        frac = (horizon - full * dtb) / dtb
        v = cum[full - 1] if full > 0 else np.zeros_like(T[0])
        if full < nt:
            v = v + frac * T[full]
        I[b] = v
    return I, dt, n4


def forward_importance(prob: dict, n_runs: int, n_per_run: int, seed0: int, grid=None,
                       options=None):
    """Forward estimate (any G): I[g][t][z][y][x] = score / weight per cell.
    Returns (I, seconds, grid cells n4)."""
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
    I = np.where((S > 0) & (Wt > 0), S / np.maximum(Wt, 1e-300), 0.0)
    return I, dt, np.asarray(q["importance"]["n"])


def training_set(I, n4, G: int):
    X = _cell_inputs(n4, G)
    Iv = np.asarray(I, float).reshape(-1)
    pos = Iv > 0
    if not pos.any():
        raise RuntimeError("importance estimate is zero everywhere: run more histories")
    y = np.log(Iv[pos]).astype(np.float32)
    wt = np.ones(int(pos.sum()), np.float32)
    return X[pos], y, wt


def _init_params(in_dim: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    H = mcdc.HIDDEN
    W1 = rng.uniform(-1, 1, (H, in_dim)) * np.sqrt(6.0 / in_dim)
    W2 = rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H)
    W3 = rng.uniform(-1, 1, (H,)) * np.sqrt(6.0 / H)
    return np.concatenate([W1.ravel(), np.full(H, 0.01), W2.ravel(), np.full(H, 0.01), W3,
                           np.zeros(1)]).astype(np.float32)


def gpu_train(X, y, wt, steps=3000, lr=3e-3, seed=1, params=None, device="cuda:0"):
    """Full-batch Adam with the library's kernels.  The output bias starts at
    the target mean.  Returns (params, loss history, seconds)."""
    import torch
    n, in_dim = X.shape
    p0 = _init_params(in_dim, seed) if params is None else np.asarray(params, np.float32).copy()
    if params is None:
        p0[-1] = np.float32(np.average(y, weights=wt))
    dev = torch.device(device)
    tX = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(dev)
    ty = torch.from_numpy(np.ascontiguousarray(y, np.float32)).to(dev)
    tw = torch.from_numpy(np.ascontiguousarray(wt, np.float32)).to(dev)
    tp = torch.from_numpy(p0).to(dev)
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


def source_log_k(prob: dict, params, ymin, ymax, n=10000, seed=3):
    """log of the mean importance exp(y) over source samples (clamped y)."""
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
    yv = np.clip(gpu_forward(params, X), ymin, ymax).astype(np.float64)
    m = yv.max()
    return float(m + np.log(np.mean(np.exp(yv - m))))


def build_ww(prob: dict, n_runs=20, n_per_run=1_000_000, seed0=W.ROOT_SEED + 1, steps=3000,
             lr=3e-3, ratio=5.0, n_max=10, method="auto", map_dims=None, grid=None,
             grid_planes=None):
    """Whole pipeline; returns (ww dict for the problem, info dict).  With
    ``map_dims`` = (nx, ny, nz, nt) the transport reads w_T from the network
    baked onto that cell-centre map instead of evaluating it at every check;
    with ``grid_planes`` = (nx, ny, nz) the windows are also checked on the
    interior planes of that grid over the outer box."""
    G = prob["sigma_t"].shape[1]
    if method == "auto":
        method = "reciprocal" if G == 1 and prob.get("detector") is not None else "forward"
    if method == "reciprocal":
        I, t_imp, n4 = reciprocal_importance(prob, n_runs, n_per_run, seed0, grid=grid)
    else:
        I, t_imp, n4 = forward_importance(prob, n_runs, n_per_run, seed0, grid=grid)
    X, y, wt = training_set(I, n4, G)
    params, losses, t_train = gpu_train(X, y, wt, steps=steps, lr=lr)
    ymin, ymax = float(y.min()), float(y.max())
    logk = source_log_k(prob, params, ymin, ymax)
    ww = dict(params=params, hidden=mcdc.HIDDEN, logk=logk, ratio=ratio, n_max=n_max,
              ymin=ymin, ymax=ymax, map=None if map_dims is None else tuple(map_dims),
              grid=None if grid_planes is None else tuple(grid_planes))
    info = dict(method=method, importance_seconds=t_imp, train_seconds=t_train,
                n_points=int(X.shape[0]), loss_first=float(losses[0]), loss_last=float(losses[-1]),
                target_var=float(np.var(y)), logk=logk, ymin=ymin, ymax=ymax)
    return ww, info


def fom_run(prob: dict, n_hist: int, seed: int, options=None, chunk: int = 100_000_000):
    """Run n_hist histories; returns (detector mean, relative error, seconds,
    counters).  The time covers the runs and the final read-back."""
    import torch
    gp = mcdc.Problem(prob, options)
    gp.run(min(n_hist, 100_000), seed + 999_999)      # warm-up; reset below
    gp.reset()
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
                  max_hist=4_000_000_000, tol=1.04, max_topups=4):
    """Pilot run -> N with the detector relative error at `target` -> run N,
    then top up (same problem, history ids continue) while the measured
    relative error exceeds tol * target.  Returns N, mean, relative error,
    seconds (all timed runs and read-backs), FOM = 1/(R^2 T) and counters."""
    import torch
    m, r, dt, _ = fom_run(prob, pilot, seed, options)
    if not (r > 0):
        raise RuntimeError("pilot run scored nothing on the detector")
    n = int(min(max_hist, max(pilot, np.ceil(pilot * (r / target) ** 2 * 1.05))))
    gp = mcdc.Problem(prob, options)
    gp.run(min(n, 100_000), seed + 999_999)            # warm-up; reset below
    gp.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, i, todo = 0, 0, n
    for _ in range(max_topups + 1):
        while todo > 0:
            k = min(todo, 100_000_000)
            gp.run(k, seed + 1000 + i)
            done += k
            todo -= k
            i += 1
        mm, rr = gp.tallies(mcdc.TALLY_DETECTOR)
        m, r = float(mm[0]), float(rr[0])
        if r <= tol * target or done >= max_hist:
            break
        todo = int(min(max_hist - done, np.ceil(done * ((r / target) ** 2 * 1.05 - 1.0))))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    c = gp.counters()
    gp.close()
    return dict(n=done, mean=m, rel_err=r, seconds=dt, fom=1.0 / (r * r * dt),
                histories_per_s=done / dt, splits=int(c["splits"]), rr_kills=int(c["rr_kills"]),
                particles=int(c["particles"]), detector_hits=int(c["detector_hits"]))
