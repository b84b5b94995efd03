"""Batched problems: each problem run inside the batch (one persistent launch
per census step, graph-replayed passes) must equal the oracle on that problem
alone, history by history, and the single-problem GPU path as well."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_04668_amd import workloads as W

from gpu_util import assert_close_sums

pytestmark = pytest.mark.gpu


def _small_batch(n_prob=7, seed=77):
    rng = np.random.default_rng(seed)
    probs = [W.batch_problem(seed + 10 + i, nt=5, n_mesh=8) for i in range(n_prob)]
    n_hist = rng.integers(1, 900, size=n_prob)
    n_hist[2] = 0                           # an empty problem
    n_hist[3] = 2048                        # exactly one chunk
    return probs, n_hist


@pytest.mark.parametrize("chunk", [0, 100])
def test_batch_matches_oracle_per_problem(chunk):
    from paper_2409_04668_amd import mcdc
    probs, n_hist = _small_batch()
    opt = mcdc.make_options(event_chunk=chunk)
    bp = mcdc.BatchProblem(probs, n_hist, opt)
    seeds = [11, 12]
    paths = []
    for s in seeds:                         # two passes: history ids continue
        bp.run(s)
        paths.append([bp.history_path(p) for p in range(len(probs))])
    for p, prob in enumerate(probs):
        r = O.OracleRun(prob, problem_id=p)
        for k, s in enumerate(seeds):
            _, ho = r.run(int(n_hist[p]), s, per_history=True)
            if n_hist[p]:
                assert np.array_equal(ho[:, 1], paths[k][p]), (p, k)
        assert_close_sums(bp.raw(p), r.tally_sum, what=f"tally p{p}")
        c = bp.counters(p)
        oc = r.counters
        for a, b in [("histories", "hist"), ("flights", "flight"), ("pieces", "piece"),
                     ("collisions", "collision"), ("leaks", "leak"), ("census_stops", "census"),
                     ("time_ends", "time_end"), ("absorptions", "absorb")]:
            assert c[a] == oc[b], (p, a, c[a], oc[b])
        assert abs(c["path"] - r.wsum["path"]) <= 1e-10 * max(r.wsum["path"], 1e-300)


def test_batch_equals_single_problem_runs():
    from paper_2409_04668_amd import mcdc
    probs, n_hist = _small_batch(5, seed=78)
    bp = mcdc.BatchProblem(probs, n_hist)
    bp.run(5)
    for p, prob in enumerate(probs):
        if not n_hist[p]:
            continue
        single = mcdc.Problem(prob, problem_id=p)
        single.set_history_scores(int(n_hist[p]))
        single.run(int(n_hist[p]), 5)
        hs = single.history_scores()
        assert np.array_equal(hs[:, 1], bp.history_path(p))
        assert_close_sums(bp.raw(p), single.raw()[0], what=f"tally p{p}")
        single.close()


def test_config5_batch_runs_and_conserves():
    """The 256-problem batch at full size: one pass, every problem's scored
    track length equals its path counter, and every history ends once."""
    from paper_2409_04668_amd import mcdc
    probs, n_hist = W.config5()
    bp = mcdc.BatchProblem(probs, n_hist)
    bp.run(20260001)
    for p in range(len(probs)):
        c = bp.counters(p)
        assert c["histories"] == n_hist[p]
        assert c["leaks"] + c["absorptions"] + c["time_ends"] == n_hist[p]
        s = bp.raw(p)
        assert abs(s.sum() - c["path"]) <= 1e-9 * max(c["path"], 1e-300)
    # sampled problems against the oracle, history by history
    for p in (0, 100, 255):
        r = O.OracleRun(probs[p], problem_id=p)
        _, ho = r.run(int(n_hist[p]), 20260001, per_history=True)
        assert np.array_equal(ho[:, 1], bp.history_path(p))
        assert_close_sums(bp.raw(p), r.tally_sum, what=f"tally p{p}")
