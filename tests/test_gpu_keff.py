"""GPU parity of the k-eigenvalue mode (power iteration on the fission
source) against the oracle: every generation's event trace and per-history
(detector score, path) bit for bit, the site counts and the site-count
estimate k_site exactly, the collision estimate k_col and the tallies to
1e-10 (the order of FP64 additions differs), counters exact; the estimate of
an infinite medium against its closed form at a size where the production
order is restored over several scan chunks; and the error paths."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04668_amd import workloads as W

from gpu_util import assert_close_sums, assert_counters, assert_traces_equal

pytestmark = pytest.mark.gpu


def _mc():
    from paper_2409_04668_amd import mcdc
    return mcdc


def _keff_parity(p, M, n_in, n_act, seed, k0=1.0, options=None, trace_cap=0):
    mc = _mc()
    gp = mc.Problem(p, options)
    orc = O.OracleRun(p)
    n_gen = n_in + n_act
    if trace_cap:
        gp.set_trace(trace_cap)
    gp.set_history_scores(n_gen * M)
    got = gp.run_keff(M, n_in, n_act, seed, k0=k0)
    ref = orc.run_keff(M, n_in, n_act, seed, k0=k0, per_history=True, trace_cap=trace_cap)
    assert np.array_equal(got["n_sites"], ref["n_sites"]), (got["n_sites"], ref["n_sites"])
    assert np.array_equal(got["k_site"], ref["k_site"])
    assert_close_sums(got["k_col"], ref["k_col"], what="k_col")
    if trace_cap:
        tg = gp.trace()
        assert len(tg) < trace_cap
        assert_traces_equal(tg, ref["trace"])
    assert np.array_equal(gp.history_scores(), ref["xh"])
    s, s2 = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")
    assert_counters(gp.counters(), orc)
    c = gp.counters()
    assert c["batches"] == n_act and c["n_hist"] == n_act * M
    # the reported results follow from the same sums
    mg, rg = gp.tallies(mc.TALLY_MESH)
    mo, ro = orc.report("mesh")
    assert_close_sums(mg, mo, rel=2e-10, what="mesh mean")
    gp.close()
    return got, ref


@pytest.mark.parametrize("implicit", [False, True])
def test_one_group_infinite_medium_parity(implicit):
    p = W.keff_infinite_medium([1.0], [[0.6]], [0.5], [1.0])
    p["implicit_capture"] = implicit
    _keff_parity(p, 2000, 2, 3, seed=81, trace_cap=400000)


def test_multigroup_infinite_medium_parity():
    st = np.array([0.8, 0.5, 0.3])
    ss = np.array([[0.6, 0.0, 0.0], [0.1, 0.3, 0.0], [0.02, 0.08, 0.15]])
    p = W.keff_infinite_medium(st, ss, [0.35, 0.05, 0.01], [0.0, 0.25, 0.75])
    _keff_parity(p, 1500, 2, 2, seed=82, trace_cap=600000)


@pytest.mark.parametrize("tile", [False, True])
def test_reflected_core_parity(tile):
    """Two groups, core and reflector, vacuum outside, 30^3 x 2 mesh bins
    (global atomics; or with an LDS hot tile over the core's centre); 10000
    histories per generation span three tiles of the site-count scan with a
    ragged last one."""
    mc = _mc()
    p = W.keff_core(nx=30)
    opt = mc.make_options(mc.SCHED_HISTORY, tile=([5, 5, 5, 0, 0], [20, 20, 20, 1, 2])) if tile \
        else mc.make_options(mc.SCHED_HISTORY)
    _keff_parity(p, 10000, 2, 3, seed=83, options=opt)


def test_pure_fissile_absorber_site_rule():
    """k_norm = nuSigma_f / Sigma_t: exactly one site per history in every
    generation, and both estimates equal k exactly."""
    p = W.keff_infinite_medium([1.0], [[0.0]], [2.5], [1.0])
    got, _ = _keff_parity(p, 3000, 0, 3, seed=84, k0=2.5)
    assert np.all(got["n_sites"] == 3000)
    assert np.all(got["k_site"] == 2.5)


def test_infinite_medium_k_at_scale():
    """5e6 histories per generation (the production-order scan runs over
    1221 tiles, two passes of its top level): the mean over 8 active
    generations of both estimates agrees with k_inf = nuSigma_f / Sigma_a."""
    mc = _mc()
    p = W.keff_infinite_medium([1.0], [[0.6]], [0.5], [1.0])
    gp = mc.Problem(p)
    M = 5_000_000
    out = gp.run_keff(M, 2, 8, seed=85)
    gp.close()
    kinf = 0.5 / 0.4
    for est in ("k_col", "k_site"):
        m, se = O.OracleRun.keff_stats(out[est], 2)
        assert abs(m - kinf) < 4.0 * se + 1e-12, (est, m, se)
        assert se < 2e-3
    # generation 0 is normalised by k0 = 1, so it makes about k_inf M sites;
    # each later one by the previous estimate, so about M
    assert abs(out["n_sites"][0] / M - kinf) < 0.02
    assert np.all(np.abs(out["n_sites"][1:].astype(float) / M - 1.0) < 0.02)


def test_keff_error_paths():
    mc = _mc()
    p = W.keff_infinite_medium([1.0], [[0.6]], [0.5], [1.0])
    gp = mc.Problem(p)
    with pytest.raises(mc.McdcError) as e:
        gp.run(100, 1)                              # fixed-source run of a fissile problem
    assert e.value.status == mc.E_STATE
    with pytest.raises(mc.McdcError) as e:
        gp.run_keff(100, 0, 0, 1)                   # no active generation
    assert e.value.status == mc.E_INVALID
    with pytest.raises(mc.McdcError) as e:
        gp.run_keff(100, 0, 2, 1, k0=1e-3)          # ~1250 sites per history: site bank overflow
    assert e.value.status == mc.E_BANK
    gp.reset()
    gp.run_keff(100, 0, 2, 1)
    with pytest.raises(mc.McdcError) as e:
        gp.run_keff(100, 0, 2, 1)                   # not fresh: ids would repeat
    assert e.value.status == mc.E_STATE
    gp.close()
    q = W.keff_infinite_medium([1.0], [[0.0]], [1e-9], [1.0])
    gq = mc.Problem(q)
    with pytest.raises(mc.McdcError) as e:
        gq.run_keff(50, 0, 2, 2)
    assert e.value.status == mc.E_EXTINCT
    gq.close()
    gh = mc.Problem(p, mc.make_options(mc.SCHED_HYBRID, event_chunk=4096))
    with pytest.raises(mc.McdcError) as e:
        gh.run_keff(100, 0, 2, 1)
    assert e.value.status == mc.E_STATE
    gh.close()
