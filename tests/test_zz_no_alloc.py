"""The MLP training entry point that allocates nothing (its scratch is a
static device array of the library) against the entry point that takes a
caller-owned scratch: two calls in a row, the second with fewer points (so
the static array still holds the first call's partial sums), give the same
parameters, Adam moments, last gradient and step count bit for bit, and the
same loss history to float-atomic summation order; a training set too large
for the static array is refused."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

IN = 5


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = np.concatenate([rng.uniform(-1, 1, (n, 4)), np.ones((n, 1))], axis=1).astype(np.float32)
    y = (np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2] - 0.5 * X[:, 3]).astype(np.float32)
    wt = rng.uniform(0.5, 2.0, n).astype(np.float32)
    return X, y, wt


def _train(noalloc, p0, X, y, wt, steps, step0=0):
    import torch
    from paper_2409_04668_amd import mcdc
    dev = torch.device("cuda:0")
    tp = torch.from_numpy(p0.copy()).to(dev)
    tX, ty, tw = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (X, y, wt))
    m = torch.zeros_like(tp)
    v = torch.zeros_like(tp)
    g = torch.zeros_like(tp)
    lh = torch.full((steps,), 7.0, dtype=torch.float32, device=dev)    # cleared by the call
    o = mcdc.TrainOpts(steps, 3e-3, 0.9, 0.999, 1e-8)
    step = C.c_int32(step0)
    n = len(X)
    if noalloc:
        st = mcdc._lib.mcdc_mlp_train_noalloc(mcdc._ptr(tp), IN, mcdc._ptr(tX), mcdc._ptr(ty),
                                               mcdc._ptr(tw), n, mcdc._ptr(m), mcdc._ptr(v),
                                               mcdc._ptr(g), C.byref(o), C.byref(step),
                                               mcdc._ptr(lh), mcdc._stream_ptr())
    else:
        scr = torch.empty(int(mcdc._lib.mcdc_mlp_scratch_bytes(IN, n)), dtype=torch.uint8, device=dev)
        st = mcdc._lib.mcdc_mlp_train(mcdc._ptr(tp), IN, mcdc._ptr(tX), mcdc._ptr(ty),
                                      mcdc._ptr(tw), n, mcdc._ptr(m), mcdc._ptr(v), mcdc._ptr(g),
                                      C.byref(o), C.byref(step), mcdc._ptr(lh), mcdc._ptr(scr),
                                      mcdc._stream_ptr())
    mcdc.check(st, "train")
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (tp, m, v, g, lh)] + [step.value]


def test_noalloc_training_matches_the_scratch_entry_point():
    from oracle import mlp as M
    p0 = M.init_params(IN, 64, seed=11)
    for n, steps, seed in ((5613, 30, 1), (777, 20, 2)):      # second call: fewer points
        X, y, wt = _data(n, seed)
        ref = _train(False, p0, X, y, wt, steps, step0=3)
        got = _train(True, p0, X, y, wt, steps, step0=3)
        # parameters, moments and the last gradient: bit for bit (the
        # gradient sums run in a fixed order)
        for a, b in zip(got[:4], ref[:4]):
            assert np.array_equal(a, b)
        # the loss history: each step's loss is summed over workgroups by
        # float atomics, whose order differs from call to call
        np.testing.assert_allclose(got[4], ref[4], rtol=1e-5)
        assert got[5] == ref[5] == 3 + steps
        assert np.all(got[4] > 0.0)                          # the loss history was written


def test_noalloc_training_refuses_more_points_than_its_scratch_holds():
    import torch
    from paper_2409_04668_amd import mcdc
    n = 58241                                                # one workgroup past the static array
    dev = torch.device("cuda:0")
    buf = torch.zeros(n * IN, dtype=torch.float32, device=dev)
    o = mcdc.TrainOpts(1, 1e-3, 0.9, 0.999, 1e-8)
    step = C.c_int32(0)
    p = mcdc._ptr(buf)
    st = mcdc._lib.mcdc_mlp_train_noalloc(p, IN, p, p, p, n, p, p, p, C.byref(o), C.byref(step),
                                          None, mcdc._stream_ptr())
    assert st == mcdc.E_INVALID
    assert b"static" in mcdc._lib.mcdc_last_error()
    assert step.value == 0
