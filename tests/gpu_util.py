"""Helpers for the GPU parity tests: run the same seeded problem through the
HIP library and through the CPU oracle and compare."""
import numpy as np

from oracle import oracle as O

INT_COUNTERS = [("hist", "histories"), ("flight", "flights"), ("piece", "pieces"),
                ("collision", "collisions"), ("absorb", "absorptions"), ("surface", "surfaces"),
                ("leak", "leaks"), ("census", "census_stops"), ("time_end", "time_ends"),
                ("split", "splits"), ("rr_kill", "rr_kills"), ("rr_survive", "rr_survivals"),
                ("cut_kill", "cutoff_kills"), ("cut_survive", "cutoff_survivals"),
                ("det_hit", "detector_hits"), ("particle", "particles"),
                ("pc_kill", "pc_kills"), ("pc_copy", "pc_copies"),
                ("surf_cross", "surf_crossings"), ("ww_plane", "ww_plane_stops")]
W_COUNTERS = [("source", "w_source"), ("leak", "w_leak"), ("absorb", "w_absorb"),
              ("time_end", "w_time_end"), ("gain", "w_gain"), ("loss", "w_loss"),
              ("path", "path")]
TRACE_FIELDS = ["hist", "tag", "seq", "type", "g", "cell", "k", "x", "y", "z", "t", "ux", "uy",
                "uz", "w", "aux"]

REL_TOL = 1e-10          # reordered FP64 sums of the same terms


def sort_trace(tr):
    return tr[np.lexsort((tr["seq"], tr["tag"], tr["hist"]))]


def assert_traces_equal(gpu, orc):
    assert len(gpu) == len(orc), (len(gpu), len(orc))
    g = sort_trace(gpu)
    o = sort_trace(orc)
    for f in TRACE_FIELDS:
        if not np.array_equal(g[f], o[f]):
            bad = np.nonzero(g[f] != o[f])[0][0]
            raise AssertionError(f"trace field {f} differs at record {bad}: gpu {g[bad]} oracle {o[bad]}")


def assert_close_sums(g, o, rel=REL_TOL, what="tally"):
    g = np.asarray(g, float)
    o = np.asarray(o, float)
    assert g.shape == o.shape
    assert np.array_equal(g == 0.0, o == 0.0), f"{what}: zero pattern differs"
    nz = o != 0.0
    if nz.any():
        err = np.max(np.abs(g[nz] - o[nz]) / np.abs(o[nz]))
        assert err <= rel, f"{what}: max rel err {err}"


def assert_counters(gc: dict, orc: "O.OracleRun", rel=REL_TOL):
    oc = orc.counters
    for ok, gk in INT_COUNTERS:
        assert gc[gk] == oc[ok], (gk, gc[gk], oc[ok])
    ow = orc.wsum
    for ok, gk in W_COUNTERS:
        a, b = gc[gk], ow[ok]
        assert abs(a - b) <= rel * max(abs(b), 1e-300) or a == b, (gk, a, b)
    assert_close_sums(gc["leak"], orc.leak, rel, "leak")
    d1, d2 = orc.detector
    assert_close_sums([gc["det_sum"], gc["det_sumsq"]], [d1, d2], rel, "detector")


def run_pair(prob, n, seed, trace_cap=0, options=None, runs=1):
    """Run `runs` consecutive runs of n histories on both sides."""
    from paper_2409_04668_amd import mcdc
    gp = mcdc.Problem(prob, options)
    orc = O.OracleRun(prob)
    traces_g, traces_o, hs_g, hs_o = [], [], [], []
    for r in range(runs):
        if trace_cap:
            gp.set_trace(trace_cap)
        gp.set_history_scores(n if n else None)
        gp.run(n, seed + r)
        to, ho = orc.run(n, seed + r, trace_cap=trace_cap, per_history=bool(n))
        if trace_cap:
            tg = gp.trace()
            assert len(tg) < trace_cap, "trace buffer too small"
            traces_g.append(tg)
            traces_o.append(to)
        if n:
            hs_g.append(gp.history_scores())
            hs_o.append(ho)
    return gp, orc, traces_g, traces_o, hs_g, hs_o


def full_parity(prob, n, seed, trace_cap=0, options=None, runs=1):
    gp, orc, tg, to, hg, ho = run_pair(prob, n, seed, trace_cap, options, runs)
    for a, b in zip(tg, to):
        assert_traces_equal(a, b)
    for a, b in zip(hg, ho):
        assert np.array_equal(a, b), np.nonzero(a != b)
    s, s2 = gp.raw()
    assert_close_sums(s, orc.tally_sum, what="tally_sum")
    assert_close_sums(s2, orc.tally_sumsq, what="tally_sumsq")
    if prob.get("collision_tally"):
        c, c2 = gp.raw_collision()
        assert_close_sums(c, orc.col_sum, what="col_sum")
        assert_close_sums(c2, orc.col_sumsq, what="col_sumsq")
    if prob.get("surface_tally") is not None:
        c, c2 = gp.raw_surface()
        assert_close_sums(c, orc.surf_sum, what="surf_sum")
        assert_close_sums(c2, orc.surf_sumsq, what="surf_sumsq")
    assert_counters(gp.counters(), orc)
    return gp, orc
