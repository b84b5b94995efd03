"""Pins of the oracle's k-eigenvalue mode (power iteration on the fission
source) against what the mathematics fixes:

* infinite homogeneous medium, one group: every source neutron's expected
  fission production is nuSigma_f / Sigma_a, so k = nuSigma_f / Sigma_a, for
  analog and implicit-capture collisions;
* infinite medium, several groups: k = nuSigma_f^T (diag Sigma_t -
  Sigma_s^T)^-1 chi, the one non-zero eigenvalue of the (rank one) fission
  matrix, cross-checked with numpy's general eigenvalue routine;
* a pure fissile absorber: each history has one collision producing exactly
  w nuSigma_f / Sigma_t / k_norm expected sites by the rule floor(x + xi), so
  with k_norm = nuSigma_f / Sigma_t every history makes exactly one site, and
  with k_norm = 1 the count is 2 or 3 with probability 1/2 each (binomial);
* the fission spectrum: sites' groups follow chi (chi-square);
* the comb, by brute force: the second generation's sources sit exactly at
  the sites floor((j + xi) S / M) of the first generation's production order,
  reconstructed from the event trace;
* tallies: only the active generations score, one batch each, and the mesh
  total equals their track length; a fixed-source run refuses fission data;
  a source that dies out is an error.  CPU only."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_2409_04668_amd import workloads as W

KEFF_TAG = 0x6B656666


def _kinf(st, ss, nf, chi):
    A = np.diag(st) - np.asarray(ss).T
    return float(np.asarray(nf) @ np.linalg.solve(A, chi))


@pytest.mark.parametrize("implicit", [False, True])
def test_one_group_infinite_medium(implicit):
    p = W.keff_infinite_medium([1.0], [[0.6]], [0.5], [1.0])
    p["implicit_capture"] = implicit
    r = O.OracleRun(p)
    out = r.run_keff(4000, 2, 40, seed=71)
    kinf = 0.5 / 0.4
    for est in ("k_col", "k_site"):
        m, se = O.OracleRun.keff_stats(out[est], 2)
        assert abs(m - kinf) < 4.0 * se, (est, m, se)
        assert se < 0.01


def test_multigroup_infinite_medium():
    st = np.array([0.8, 0.5, 0.3])
    ss = np.array([[0.6, 0.0, 0.0],           # rows: from-group (0 slowest)
                   [0.1, 0.3, 0.0],
                   [0.02, 0.08, 0.15]])
    nf = np.array([0.35, 0.05, 0.01])
    chi = np.array([0.0, 0.25, 0.75])
    kinf = _kinf(st, ss, nf, chi)
    F = np.linalg.solve(np.diag(st) - ss.T, np.outer(chi, nf))   # fission matrix
    assert abs(max(np.linalg.eigvals(F).real) - kinf) < 1e-12
    p = W.keff_infinite_medium(st, ss, nf, chi)
    r = O.OracleRun(p)
    out = r.run_keff(4000, 3, 40, seed=72)
    m, se = O.OracleRun.keff_stats(out["k_col"], 3)
    assert abs(m - kinf) < 4.0 * se, (m, se, kinf)
    m2, se2 = O.OracleRun.keff_stats(out["k_site"], 3)
    assert abs(m2 - kinf) < 4.0 * se2, (m2, se2, kinf)


def test_site_count_rule_pure_fissile_absorber():
    p = W.keff_infinite_medium([1.0], [[0.0]], [2.5], [1.0])
    M = 2000
    # k_norm = 2.5: every collision yields floor(1 + xi) = 1 site exactly
    r = O.OracleRun(p)
    out = r.run_keff(M, 0, 3, seed=73, k0=2.5)
    assert np.all(out["n_sites"] == M)
    assert np.all(out["k_site"] == 2.5) and np.all(out["k_col"] == 2.5)
    # k_norm = 1: 2 or 3 sites per history, 3 with probability 1/2
    r = O.OracleRun(p)
    out = r.run_keff(M, 0, 1, seed=74, k0=1.0, trace_cap=10 * M)
    tr = out["trace"]
    n = tr["aux"][tr["type"] == O.EV["fission"]]
    assert n.size == M and set(np.unique(n)) <= {2.0, 3.0}
    assert int(n.sum()) == int(out["n_sites"][0])
    k3 = int(np.sum(n == 3.0))
    assert abs(k3 - M / 2) < 4.0 * math.sqrt(M / 4)


def test_site_groups_follow_the_fission_spectrum():
    chi = np.array([0.15, 0.35, 0.5])
    st = np.array([1.0, 1.0, 1.0])
    ss = np.zeros((3, 3))
    p = W.keff_infinite_medium(st, ss, [1.0, 1.0, 1.0], chi)
    M = 20000
    r = O.OracleRun(p)
    out = r.run_keff(M, 0, 1, seed=75, src_out=True)
    g = out["src"][:, 3].astype(int)
    counts = np.bincount(g, minlength=3)
    chi2 = np.sum((counts - M * chi) ** 2 / (M * chi))
    assert stats.chi2.sf(chi2, 2) > 1e-3, (counts, chi2)


def test_comb_by_brute_force():
    """Rebuild generation 0's sites (position, in production order) from the
    fission records of the trace and pick generation 1's sources with the
    comb; every source record of generation 1 must sit at its site."""
    p = W.keff_core(nx=3)
    M, seed = 300, 76
    r = O.OracleRun(p)
    out = r.run_keff(M, 0, 2, seed=seed, trace_cap=400000)
    tr = out["trace"]
    tr = tr[np.lexsort((tr["seq"], tr["tag"], tr["hist"]))]
    fis = tr[(tr["type"] == O.EV["fission"]) & (tr["hist"] < M)]
    sites = []
    for rec in fis:
        sites += [(rec["x"], rec["y"], rec["z"])] * int(rec["aux"])
    S = len(sites)
    assert S == int(out["n_sites"][0])
    xi = O.uniform(seed, M, 0, KEFF_TAG, 0)
    src = tr[(tr["hist"] >= M) & (tr["seq"] == 0)]
    assert len(src) == M
    assert np.all(np.isin(src["type"], [O.EV["source"], O.EV["leak"]]))
    for j, rec in enumerate(src):
        assert rec["hist"] == M + j
        idx = min(int(math.floor((j + xi) * S / M)), S - 1)
        assert (rec["x"], rec["y"], rec["z"]) == sites[idx], j
        assert rec["t"] == 0.0 and rec["w"] == 1.0


def test_only_active_generations_score():
    p = W.keff_core(nx=4)
    M, n_in, n_act = 500, 2, 3
    r = O.OracleRun(p)
    out = r.run_keff(M, n_in, n_act, seed=77, per_history=True)
    assert int(r.R.batches_done) == n_act and r.n_hist == M * n_act
    path_active = out["xh"][n_in * M:, 1].sum()
    assert abs(r.tally_sum.sum() - path_active) <= 1e-12 * path_active
    d1, d2 = r.detector
    xh = out["xh"][n_in * M:, 0]
    assert abs(d1 - xh.sum()) <= 1e-12 * max(xh.sum(), 1e-300)
    mean, rel = r.report("mesh")
    assert np.all(np.isfinite(rel))


def test_fixed_source_run_refuses_fission_and_extinction_is_an_error():
    p = W.keff_infinite_medium([1.0], [[0.6]], [0.5], [1.0])
    with pytest.raises(O.OracleError) as e:
        O.run(p, 10, seed=1)
    assert e.value.status == -1
    q = W.keff_infinite_medium([1.0], [[0.0]], [1e-9], [1.0])
    with pytest.raises(O.OracleError) as e:
        O.OracleRun(q).run_keff(50, 0, 2, seed=2)
    assert e.value.status == O.E_EXTINCT


def test_reflected_core_is_below_its_infinite_medium_value():
    p = W.keff_core(nx=3)
    kinf = _kinf(p["sigma_t"][0], p["sigma_s"][0], p["nu_sigma_f"][0], p["chi"][0])
    r = O.OracleRun(p)
    out = r.run_keff(3000, 5, 10, seed=78)
    m, se = O.OracleRun.keff_stats(out["k_col"], 5)
    ms, ses = O.OracleRun.keff_stats(out["k_site"], 5)
    assert m < kinf - 5 * se                       # leakage
    assert abs(m - ms) < 4.0 * math.hypot(se, ses)  # two estimators of one k
