"""Pins of the oracle's statistical error: the standard errors that the
figure of merit 1/(R^2 T) rests on (R = standard error / mean).

A pure absorber hit by a beam along +x is a problem whose per-history score
distribution is known in closed form: the flight length s ~ Exp(Sigma), the
detector covering the slab [0, L] scores x = min(s, L), and mesh bin [a, b]
scores clip(s - a, 0, b - a).  Every moment E[x^k] = int k u^(k-1) P(s > u) du
follows by quadrature of exp(-Sigma u), so the true standard error of the
mean, sqrt(Var[x] / N), is known.  The estimators are pinned two ways:

* against that closed form directly: the detector's per-history estimator
  and the mesh's batch-means estimator (1000 batches, unequal sizes) must
  reproduce sqrt(Var[x] / N) to within their own sampling error;
* by replication: over many independent seeds the z-scores (mean - truth) /
  standard error must have unit variance, inside chi-square bounds.

A standard error inflated or deflated by a constant factor (sqrt(B), sqrt(2),
N / (N - 1) applied twice, a dropped batch) fails one of them.  The
reported values (mean / (volume x time width), rel = se / mean) are checked
on a hand-computed case.  CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import oracle as O
from paper_2409_04668_amd import workloads as W

SIG, L = 1.0, 2.0
BIG = 1e9


def _absorber_beam(nx=4, n_batches=20, length=L):
    p = W.slab_problem(sigma_t=SIG, c=0.0, length=length, t_end=BIG, nx=nx, nt=1,
                       detector=(0.0, length))
    p["source"]["isotropic"] = False
    p["source"]["dir"] = np.array([1.0, 0.0, 0.0])
    p["n_batches"] = n_batches
    return p


def _moments(a, b, kmax=4):
    """E[x^k], k = 1..kmax, for x = clip(s - a, 0, b - a), s ~ Exp(SIG)."""
    out = []
    for k in range(1, kmax + 1):
        f = lambda u, k=k: k * u ** (k - 1) * math.exp(-SIG * (a + u))
        out.append(integrate.quad(f, 0.0, b - a, epsabs=1e-14, epsrel=1e-12)[0])
    return out


def _var_and_se_of_sd(a, b, n):
    """Variance of the per-history score, and the standard error of a sample
    standard deviation over n scores (delta method: sd(s^2) / (2 sigma^2))."""
    m1, m2, m3, m4 = _moments(a, b)
    var = m2 - m1 * m1
    mu4 = m4 - 4 * m3 * m1 + 6 * m2 * m1 * m1 - 3 * m1 ** 4
    return m1, var, math.sqrt((mu4 - var * var) / n) / (2 * var)


def test_moment_quadrature_matches_closed_form():
    """The quadrature behind the pins reproduces the textbook first two
    moments of min(s, L): (1 - e^-SL)/S and 2 (1 - e^-SL (1 + SL)) / S^2."""
    m1, m2, _, _ = _moments(0.0, L)
    e = math.exp(-SIG * L)
    assert abs(m1 - (1 - e) / SIG) < 1e-12
    assert abs(m2 - 2 * (1 - e * (1 + SIG * L)) / SIG ** 2) < 1e-12


def test_detector_standard_error_matches_closed_form():
    N = 200_000
    r = O.run(_absorber_beam(), N, seed=2101)
    m, se = r.detector_stats()
    mu, var, rel_se_of_sd = _var_and_se_of_sd(0.0, L, N)
    truth = math.sqrt(var / N)
    assert abs(m - mu) < 4.0 * truth
    # the estimated standard error is the true one within its own sampling error
    assert abs(se / truth - 1.0) < 5.0 * rel_se_of_sd, (se, truth, rel_se_of_sd)
    # and the reported relative error is that standard error over the mean
    mean, rel = r.report("detector")
    assert mean[0] == m and rel[0] == se / m


def test_mesh_batch_standard_error_matches_closed_form():
    """Batch means over 1000 unequal batches (N is not a multiple of B): per
    bin, the weighted batch estimator reproduces sqrt(Var[x_bin] / N)."""
    N, B, nx = 200_037, 1000, 4
    r = O.run(_absorber_beam(nx=nx, n_batches=B), N, seed=2102)
    assert int(r.R.batches_done) == B
    mean, se = r.mesh_stats()
    assert mean.shape == (nx,)
    # relative sampling error of a batch-means standard deviation with B - 1
    # degrees of freedom (batch sums of ~200 histories are close to normal)
    tol = 5.0 / math.sqrt(2.0 * (B - 1))
    dx = L / nx
    for i in range(nx):
        mu, var, _ = _var_and_se_of_sd(i * dx, (i + 1) * dx, N)
        truth = math.sqrt(var / N)
        assert abs(mean[i] - mu) < 4.0 * truth, (i, mean[i], mu, truth)
        assert abs(se[i] / truth - 1.0) < tol, (i, se[i], truth)


def test_replicated_z_scores_have_unit_variance():
    """Independent seeds: (mean - truth) / se must scatter with unit variance.
    Detector (per-history estimator) and every mesh bin (50 batches, whose
    z-scores follow Student's t with 49 degrees of freedom)."""
    K, N, B, nx = 200, 4000, 50, 4
    p = _absorber_beam(nx=nx, n_batches=B)
    zd, zm = [], []
    for k in range(K):
        r = O.run(p, N, seed=3000 + k)
        m, se = r.detector_stats()
        mu, _, _ = _var_and_se_of_sd(0.0, L, N)
        zd.append((m - mu) / se)
        mm, sm = r.mesh_stats()
        zm.append([(mm[i] - _moments(i * L / nx, (i + 1) * L / nx, 1)[0]) / sm[i]
                   for i in range(nx)])
    zd = np.array(zd)
    zm = np.array(zm)
    lo, hi = stats.chi2.ppf([0.0005, 0.9995], K - 1) / (K - 1)
    assert lo < np.var(zd, ddof=1) < hi, np.var(zd, ddof=1)
    assert abs(np.mean(zd)) < 4.0 / math.sqrt(K)
    t_var = (B - 1) / (B - 3)                       # variance of Student's t
    for i in range(nx):
        v = np.var(zm[:, i], ddof=1) / t_var
        # t is slightly heavy-tailed: widen the chi-square band by its kurtosis
        assert 0.8 * lo < v < 1.2 * hi, (i, v)


def test_report_divides_by_bin_volume_and_time_width():
    """mean / (dx dy dz dt) on a mesh with every kind of axis: bounded x and
    y, an unbounded z (not cut), and time."""
    p = W.slab_problem(sigma_t=0.5, c=0.5, length=4.0, t_end=6.0, nx=4, nt=3, detector=None)
    p["outer_lo"] = np.array([0.0, -1.0, -W.INF])
    p["outer_hi"] = np.array([4.0, 1.0, W.INF])
    p["bc"][2:4] = W.REFLECTIVE
    p["mesh"]["lo"] = np.array([0.0, -1.0, -W.INF, 0.0])
    p["mesh"]["hi"] = np.array([4.0, 1.0, W.INF, 6.0])
    p["mesh"]["n"] = np.array([4, 5, 1, 3], np.int32)
    r = O.run(p, 3000, seed=2103)
    mean, se = r.mesh_stats()
    rep, rel = r.report("mesh")
    vol = 1.0 * 0.4 * 2.0                           # dx = 1, dy = 0.4, dt = 2
    assert np.array_equal(rep, mean / vol)
    nz = mean > 0
    assert np.array_equal(rel[nz], se[nz] / mean[nz])
    assert np.all(rel[~nz] == 0.0)


def test_report_edge_cases():
    """Fewer histories than batches: empty batches are not counted; one
    history gives no error estimate (NaN); leakage carries no error."""
    p = _absorber_beam(nx=2, n_batches=20)
    r = O.run(p, 1, seed=2104)
    assert int(r.R.batches_done) == 1
    _, rel = r.report("mesh")
    assert np.all(np.isnan(rel))
    _, rd = r.report("detector")
    assert np.isnan(rd[0])
    r.run(6, seed=2105)                             # 6 histories over 20 batches
    assert int(r.R.batches_done) == 7
    m, rel = r.report("mesh")
    assert np.all(np.isfinite(rel[m > 0]))
    lk, lrel = r.report("leakage")
    assert np.array_equal(lk, r.leak / 7.0) and np.all(np.isnan(lrel))
