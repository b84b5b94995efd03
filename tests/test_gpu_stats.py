"""Reported results on the GPU: mcdc_get_tallies (mean and relative error of
every tally kind) against the oracle's definition of the run's output, the
device read-back against the host read-back, and the cancel word.

The oracle's side is OracleRun.report, pinned on the CPU against closed-form
variances and by replication (tests/test_oracle_stats.py).  The library's
tally sums S and S2 match the oracle's to 1e-10 relative (only the order of
FP64 additions differs); the tolerance of each reported value is that
difference carried through the definition of the value."""
import threading
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04668_amd import workloads as W

from gpu_util import assert_close_sums

pytestmark = pytest.mark.gpu

REL = 1e-10


def _mc():
    from paper_2409_04668_amd import mcdc
    return mcdc


def _problem():
    p = W.config1()
    p["collision_tally"] = True
    p["surface_tally"] = dict(axis=0, pos=5.0)
    p["n_batches"] = 7
    return p


def _rel_tol(s, s2, N, B, rel_o):
    """Bound on |rel_gpu - rel_oracle| when S and S2 each differ by at most
    REL relative: the numerator S2 - S^2/N moves by at most REL (S2 + 2 S^2/N)
    (bound a); rel = sqrt(numerator / ((B - 1) N)) / m then moves by about
    rel (a / (2 numerator) + REL) where the numerator is well above a, and by
    at most sqrt(a / ((B - 1) N)) / m anywhere (|sqrt x - sqrt y| <=
    sqrt |x - y|).  Doubled for the rounding of the final operations."""
    m = s / N
    a = 2.0 * REL * (s2 + 2.0 * s * s / N)
    num = s2 - s * s / N
    with np.errstate(divide="ignore", invalid="ignore"):
        lin = rel_o * (a / (2.0 * np.maximum(num, 1e-300)) + 2.0 * REL)
        sq = np.sqrt(a / ((B - 1.0) * N)) / np.where(m > 0, m, 1.0)
    return np.where(num > 1e4 * a, lin, sq) + 1e-15


def _check_kind(gp, orc, kind_name, kind, sums):
    mc = _mc()
    mean_g, rel_g = gp.tallies(kind)
    mean_o, rel_o = orc.report(kind_name)
    # the device read-back is the same arithmetic: identical bits
    dm, dr = gp.tallies_device(kind)
    assert np.array_equal(dm.cpu().numpy(), mean_g, equal_nan=True), kind_name
    assert np.array_equal(dr.cpu().numpy(), rel_g, equal_nan=True), kind_name
    dm2, none = gp.tallies_device(kind, with_rel=False)
    assert none is None and np.array_equal(dm2.cpu().numpy(), mean_g)
    assert_close_sums(mean_g, mean_o, rel=2 * REL, what=f"{kind_name} mean")
    assert np.array_equal(np.isnan(rel_g), np.isnan(rel_o)), f"{kind_name}: NaN pattern"
    ok = ~np.isnan(rel_o)
    if not ok.any():
        return
    if kind == mc.TALLY_DETECTOR:
        s, s2 = orc.detector
        N = float(orc.n_hist)
        # per-history estimator: the numerator is X2/N - m^2 (same bound with B - 1 = N - 1
        # and S2 scaled by 1/N)
        tol = _rel_tol(np.array([s]), np.array([s2]), N, N, rel_o)
    else:
        s, s2 = sums
        tol = _rel_tol(s, s2, float(orc.n_hist), float(orc.R.batches_done), rel_o)
    diff = np.abs(rel_g - rel_o)
    assert np.all(diff[ok] <= tol[ok]), (kind_name, np.max(diff[ok] - tol[ok]))
    # and rel is zero exactly where the mean is zero
    assert np.array_equal(rel_g[ok] == 0.0, rel_o[ok] == 0.0), kind_name


@pytest.mark.parametrize("sched", ["history", "hybrid", "event"])
def test_reported_results_match_oracle(sched):
    """One history (every relative error NaN), then fewer histories than
    batches (empty batches skipped), then unequal batches (1003 histories in
    7 batches) and a further run accumulated on top: after each run every
    kind of result (mesh, collision estimator, surface current, detector,
    leakage) matches the oracle's report."""
    mc = _mc()
    opt = {"history": mc.make_options(mc.SCHED_HISTORY),
           "hybrid": mc.make_options(mc.SCHED_HYBRID, event_chunk=4096),
           "event": mc.make_options(mc.SCHED_EVENT, event_chunk=4096)}[sched]
    p = _problem()
    gp = mc.Problem(p, opt)
    orc = O.OracleRun(p)
    for n, seed in ((1, 11), (5, 12), (1003, 13), (2000, 14)):
        gp.run(n, seed)
        orc.run(n, seed)
        s, s2 = gp.raw()
        assert_close_sums(s, orc.tally_sum, what="tally_sum")
        assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")
        c = gp.counters()
        assert c["batches"] == orc.R.batches_done and c["n_hist"] == orc.n_hist
        _check_kind(gp, orc, "mesh", mc.TALLY_MESH, (orc.tally_sum, orc.tally_sumsq))
        _check_kind(gp, orc, "collision", mc.TALLY_COLLISION, (orc.col_sum, orc.col_sumsq))
        _check_kind(gp, orc, "surface", mc.TALLY_SURFACE, (orc.surf_sum, orc.surf_sumsq))
        _check_kind(gp, orc, "detector", mc.TALLY_DETECTOR, None)
        _check_kind(gp, orc, "leakage", mc.TALLY_LEAKAGE, None)
    gp.close()


def test_reported_results_duct_full_mesh():
    """The duct's 7.2e6-bin mesh with its detector, 20 batches."""
    mc = _mc()
    p = W.config2()
    gp = mc.Problem(p, mc.make_options(mc.SCHED_HYBRID, event_chunk=1 << 16))
    orc = O.OracleRun(p)
    gp.run(20000, 31)
    orc.run(20000, 31)
    _check_kind(gp, orc, "mesh", mc.TALLY_MESH, (orc.tally_sum, orc.tally_sumsq))
    _check_kind(gp, orc, "detector", mc.TALLY_DETECTOR, None)
    _check_kind(gp, orc, "leakage", mc.TALLY_LEAKAGE, None)
    gp.close()


def test_results_need_histories_and_the_right_kind():
    mc = _mc()
    p = W.config1()
    gp = mc.Problem(p)
    with pytest.raises(mc.McdcError) as e:
        gp.tallies(mc.TALLY_MESH)
    assert e.value.status == mc.E_STATE
    gp.run(10, 1)
    with pytest.raises(mc.McdcError) as e:
        gp.tallies(mc.TALLY_COLLISION)          # created without the collision estimator
    assert e.value.status == mc.E_STATE
    with pytest.raises(mc.McdcError) as e:
        gp.tallies_device(mc.TALLY_SURFACE)
    assert e.value.status == mc.E_STATE
    gp.close()


# ---- cancel word --------------------------------------------------------------

@pytest.mark.parametrize("sched", ["history", "hybrid"])
def test_cancel_set_before_the_run(sched):
    """With the word set beforehand, the persistent kernel reads it on its
    first loop turn and every work-item leaves before starting a history; the
    run returns MCDC_E_CANCELLED and the status sticks until a reset.  Then the
    handle runs normally again, history for history as the oracle."""
    mc = _mc()
    opt = (mc.make_options(mc.SCHED_HISTORY) if sched == "history"
           else mc.make_options(mc.SCHED_HYBRID, event_chunk=4096))
    p = W.config1()
    gp = mc.Problem(p, opt)
    gp.set_cancel(True)
    with pytest.raises(mc.McdcError) as e:
        gp.run(5000, 3)
    assert e.value.status == mc.E_CANCELLED
    c = gp.counters()
    assert c["status"] == mc.E_CANCELLED
    assert c["particles"] == 0 and c["flights"] == 0       # no source was sampled
    with pytest.raises(mc.McdcError) as e:
        gp.tallies(mc.TALLY_DETECTOR)
    assert e.value.status == mc.E_CANCELLED
    gp.set_cancel(False)
    gp.reset()
    gp.set_history_scores(3000)
    gp.run(3000, 4)
    orc = O.OracleRun(p)
    _, ho = orc.run(3000, 4, per_history=True)
    assert np.array_equal(gp.history_scores(), ho)
    assert gp.counters()["status"] == 0
    gp.close()


def test_cancel_while_running():
    """The word set from another thread while a long history-schedule launch
    runs (2e9 duct histories, about a second): the launch ends early, with
    fewer histories than asked and the cancelled status."""
    import torch
    mc = _mc()
    p = W.config2()
    p["n_batches"] = 1
    p["detector"] = None
    gp = mc.Problem(p, mc.make_options(mc.SCHED_HISTORY))
    n = 2_000_000_000
    gp.run(n, 5)                      # enqueued; the launch runs asynchronously

    def later():
        time.sleep(0.1)
        gp.set_cancel(True)

    th = threading.Thread(target=later)
    t0 = time.perf_counter()
    th.start()
    th.join()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    c = gp.counters()
    print(f"cancelled after {dt:.3f} s: {c['histories']} of {n} histories")
    assert c["status"] == mc.E_CANCELLED
    assert 0 < c["histories"] < n
    gp.close()


def test_cancel_batched_run():
    mc = _mc()
    probs = [W.batch_problem(i) for i in range(4)]
    bp = mc.BatchProblem(probs, [20000, 5000, 100, 3000])
    bp.set_cancel(True)
    with pytest.raises(mc.McdcError) as e:
        bp.run(7)
    assert e.value.status == mc.E_CANCELLED
    for i in range(4):
        c = bp.counters(i)
        assert c["status"] == mc.E_CANCELLED
    bp.close()


def test_cancel_keff_run():
    """The word set before a k-eigenvalue run: the first generation's launch
    leaves at once, nothing is combed from the sites it did not make, the run
    returns MCDC_E_CANCELLED; after a reset the same handle runs the
    generations as an uncancelled handle does."""
    mc = _mc()
    p = W.keff_infinite_medium([1.0], [[0.6]], [0.5], [1.0])
    ref = mc.Problem(p)
    want = ref.run_keff(2000, 1, 3, seed=91)
    ref.close()
    gp = mc.Problem(p)
    gp.set_cancel(True)
    with pytest.raises(mc.McdcError) as e:
        gp.run_keff(2000, 1, 3, seed=91)
    assert e.value.status == mc.E_CANCELLED
    c = gp.counters()
    assert c["flights"] == 0 and c["n_hist"] == 0
    gp.set_cancel(False)
    gp.reset()
    got = gp.run_keff(2000, 1, 3, seed=91)
    # the site counts, and so k_site, are exact; k_col sums per-workgroup
    # partials in the order the work-items finish
    for k in ("k_site", "n_sites"):
        assert np.array_equal(got[k], want[k]), k
    np.testing.assert_allclose(got["k_col"], want["k_col"], rtol=1e-12)
    gp.close()

