"""ctypes front end of the CPU oracle.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this module.  It marshals the problem dicts built by
``paper_2409_04668_amd.workloads`` into the oracle's own C structs (declared
again here, independently of the GPU library's header) and returns numpy
results.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wno-unused-function"]

NCOUNT = 20
NWSUM = 7
COUNTER_NAMES = ["hist", "flight", "piece", "collision", "absorb", "surface", "leak",
                 "census", "time_end", "split", "rr_kill", "rr_survive", "cut_kill",
                 "cut_survive", "det_hit", "particle", "pc_kill", "pc_copy", "surf_cross",
                 "ww_plane"]
WSUM_NAMES = ["source", "leak", "absorb", "time_end", "gain", "loss", "path"]

EV = dict(source=0, scatter=1, absorb=2, surface=3, leak=4, census=5, time_end=6, split=7,
          roulette_kill=8, roulette_survive=9, cutoff_kill=10, cutoff_survive=11, pc_kill=12,
          pc_keep=13, ww_plane=14, fission=15)
E_EXTINCT = -9


def build(force: bool = True) -> str:
    src = os.path.join(HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


D3 = C.c_double * 3
D4 = C.c_double * 4
I4 = C.c_int32 * 4
I6 = C.c_int32 * 6
PD = C.POINTER(C.c_double)
PI = C.POINTER(C.c_int32)
PF = C.POINTER(C.c_float)


class OrcProblem(C.Structure):
    _fields_ = [
        ("outer_lo", D3), ("outer_hi", D3), ("bc", I6),
        ("n_boxes", C.c_int32), ("box_lo", PD), ("box_hi", PD), ("box_mat", PI),
        ("background_mat", C.c_int32), ("n_mat", C.c_int32), ("G", C.c_int32),
        ("sigma_t", PD), ("sigma_s", PD), ("speed", PD),
        ("src_box", C.c_int32), ("src_lo", D3), ("src_hi", D3), ("src_t0", C.c_double),
        ("src_t1", C.c_double), ("src_isotropic", C.c_int32), ("src_dir", D3),
        ("src_group", C.c_int32),
        ("mesh_lo", D4), ("mesh_hi", D4), ("mesh_n", I4), ("mesh_per_group", C.c_int32),
        ("n_census", C.c_int32), ("census", PD),
        ("implicit_capture", C.c_int32), ("w_cut", C.c_double), ("w_surv", C.c_double),
        ("has_detector", C.c_int32), ("det_lo", D3), ("det_hi", D3),
        ("imp_on", C.c_int32), ("imp_n", I4),
        ("ww_on", C.c_int32), ("ww_hidden", C.c_int32), ("ww_nmax", C.c_int32),
        ("ww_params", PF), ("ww_ymin", C.c_float), ("ww_ymax", C.c_float),
        ("ww_logk", C.c_double), ("ww_ratio", C.c_double), ("ww_map_n", I4),
        ("ww_grid_n", C.c_int32 * 3),
        ("col_tally", C.c_int32), ("surf_on", C.c_int32), ("surf_axis", C.c_int32),
        ("surf_pos", C.c_double), ("pc_on", C.c_int32), ("pc_target", C.c_double),
        ("n_batches", C.c_int32), ("max_events", C.c_int64), ("stack_cap", C.c_int32),
        ("problem_id", C.c_uint32), ("nu_sigma_f", PD), ("chi", PD),
    ]


class OrcKeff(C.Structure):
    _fields_ = [("M", C.c_uint64), ("n_inactive", C.c_int32), ("n_active", C.c_int32),
                ("k0", C.c_double), ("k_col", PD), ("k_site", PD),
                ("n_sites", C.POINTER(C.c_uint64)), ("src_out", PD)]


class OrcTraceRec(C.Structure):
    _fields_ = [("hist", C.c_uint64), ("tag", C.c_uint32), ("seq", C.c_uint32),
                ("type", C.c_int32), ("g", C.c_int32), ("cell", C.c_int32), ("k", C.c_uint32),
                ("x", C.c_double), ("y", C.c_double), ("z", C.c_double), ("t", C.c_double),
                ("ux", C.c_double), ("uy", C.c_double), ("uz", C.c_double), ("w", C.c_double),
                ("aux", C.c_double)]


TRACE_DTYPE = np.dtype([("hist", "<u8"), ("tag", "<u4"), ("seq", "<u4"), ("type", "<i4"),
                        ("g", "<i4"), ("cell", "<i4"), ("k", "<u4"), ("x", "<f8"), ("y", "<f8"),
                        ("z", "<f8"), ("t", "<f8"), ("ux", "<f8"), ("uy", "<f8"), ("uz", "<f8"),
                        ("w", "<f8"), ("aux", "<f8")])
assert TRACE_DTYPE.itemsize == C.sizeof(OrcTraceRec)


class OrcResult(C.Structure):
    _fields_ = [("tally_batch", PD), ("tally_sum", PD), ("tally_sumsq", PD),
                ("col_batch", PD), ("col_sum", PD), ("col_sumsq", PD),
                ("surf_batch", PD), ("surf_sum", PD), ("surf_sumsq", PD),
                ("det", C.c_double * 2), ("leak", C.c_double * 6), ("wsum", C.c_double * NWSUM),
                ("cnt", C.c_uint64 * NCOUNT), ("imp_score", PD), ("imp_weight", PD),
                ("hist_xh", PD), ("trace", C.POINTER(OrcTraceRec)), ("trace_cap", C.c_int64),
                ("trace_n", C.c_int64), ("batches_done", C.c_int64), ("hist_done", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_run.argtypes = [C.POINTER(OrcProblem), C.c_uint64, C.c_uint64, C.c_uint64,
                              C.POINTER(OrcResult)]
        L.orc_run.restype = C.c_int
        L.orc_run_keff.argtypes = [C.POINTER(OrcProblem), C.c_uint64, C.POINTER(OrcKeff),
                                   C.POINTER(OrcResult)]
        L.orc_run_keff.restype = C.c_int
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.orc_philox4x32_10.restype = None
        L.orc_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_log.argtypes = [C.c_double]
        L.orc_log.restype = C.c_double
        L.orc_exp.argtypes = [C.c_double]
        L.orc_exp.restype = C.c_double
        L.orc_directions.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, PD]
        L.orc_directions.restype = C.c_uint32
        L.orc_mlp_f32.argtypes = [PF, C.c_int32, C.c_int32, PF]
        L.orc_mlp_f32.restype = C.c_float
        L.orc_score_segment.argtypes = [C.POINTER(OrcProblem), PD, PD, C.c_double, C.c_double,
                                        C.c_double, C.c_int32, PD]
        L.orc_score_segment.restype = C.c_int64
        L.orc_ww_map.argtypes = [C.POINTER(OrcProblem), PD]
        L.orc_ww_map.restype = C.c_int64
        L.orc_ww_map_cell.argtypes = [C.POINTER(OrcProblem), PD, C.c_double, C.c_int32]
        L.orc_ww_map_cell.restype = C.c_int64
        _lib = L
    return _lib


def _pd(a):
    return a.ctypes.data_as(PD)


class _Problem:
    """Holds the C struct and keeps the numpy buffers it points to alive."""

    def __init__(self, prob: dict, problem_id: int = 0):
        self.keep = []
        s = OrcProblem()

        def arr(x, dt):
            a = np.ascontiguousarray(np.asarray(x, dtype=dt))
            self.keep.append(a)
            return a

        s.outer_lo = D3(*[float(v) for v in prob["outer_lo"]])
        s.outer_hi = D3(*[float(v) for v in prob["outer_hi"]])
        s.bc = I6(*[int(v) for v in prob["bc"]])
        nb = int(np.asarray(prob["box_mat"]).size)
        s.n_boxes = nb
        blo = arr(np.asarray(prob["box_lo"], float).reshape(-1, 3) if nb else np.zeros((1, 3)), np.float64)
        bhi = arr(np.asarray(prob["box_hi"], float).reshape(-1, 3) if nb else np.zeros((1, 3)), np.float64)
        bm = arr(prob["box_mat"] if nb else np.zeros(1), np.int32)
        s.box_lo, s.box_hi, s.box_mat = _pd(blo), _pd(bhi), bm.ctypes.data_as(PI)
        s.background_mat = int(prob["background_mat"])
        st = arr(prob["sigma_t"], np.float64)
        M, G = st.shape
        s.n_mat, s.G = M, G
        ss = arr(np.asarray(prob["sigma_s"], float).reshape(M, G, G), np.float64)
        sp = arr(prob["speed"], np.float64)
        s.sigma_t, s.sigma_s, s.speed = _pd(st), _pd(ss), _pd(sp)
        src = prob["source"]
        s.src_box = 1 if src["kind"] == "box" else 0
        s.src_lo = D3(*[float(v) for v in src["lo"]])
        s.src_hi = D3(*[float(v) for v in src["hi"]])
        s.src_t0, s.src_t1 = float(src["t0"]), float(src["t1"])
        s.src_isotropic = 1 if src["isotropic"] else 0
        s.src_dir = D3(*[float(v) for v in src["dir"]])
        s.src_group = int(src["group"])
        m = prob["mesh"]
        s.mesh_lo = D4(*[float(v) for v in m["lo"]])
        s.mesh_hi = D4(*[float(v) for v in m["hi"]])
        s.mesh_n = I4(*[int(v) for v in m["n"]])
        s.mesh_per_group = 1 if m["per_group"] else 0
        cen = arr(prob["census"], np.float64)
        s.n_census, s.census = cen.size, _pd(cen)
        s.implicit_capture = 1 if prob["implicit_capture"] else 0
        s.w_cut, s.w_surv = float(prob["w_cut"]), float(prob["w_surv"])
        det = prob.get("detector")
        s.has_detector = 1 if det is not None else 0
        if det is not None:
            s.det_lo = D3(*[float(v) for v in det["lo"]])
            s.det_hi = D3(*[float(v) for v in det["hi"]])
        imp = prob.get("importance")
        s.imp_on = 1 if imp is not None else 0
        if imp is not None:
            s.imp_n = I4(*[int(v) for v in imp["n"]])
        ww = prob.get("ww")
        s.ww_on = 1 if ww is not None else 0
        if ww is not None:
            prm = arr(ww["params"], np.float32)
            s.ww_params = prm.ctypes.data_as(PF)
            s.ww_hidden = int(ww.get("hidden", 64))
            s.ww_nmax = int(ww.get("n_max", 10))
            s.ww_logk = float(ww["logk"])
            s.ww_ratio = float(ww.get("ratio", 5.0))
            s.ww_ymin = float(ww.get("ymin", -3.0e38))
            s.ww_ymax = float(ww.get("ymax", 3.0e38))
            if ww.get("map") is not None:
                s.ww_map_n = I4(*[int(v) for v in ww["map"]])
            if ww.get("grid") is not None:
                s.ww_grid_n = (C.c_int32 * 3)(*[int(v) for v in ww["grid"]])
        s.col_tally = 1 if prob.get("collision_tally") else 0
        sf = prob.get("surface_tally")
        s.surf_on = 1 if sf is not None else 0
        if sf is not None:
            s.surf_axis = int(sf["axis"])
            s.surf_pos = float(sf["pos"])
        pc = prob.get("population_control")
        s.pc_on = 1 if pc is not None else 0
        s.pc_target = float(pc["target"]) if pc is not None else 0.0
        s.n_batches = int(prob["n_batches"])
        s.max_events = int(prob["max_events"])
        s.stack_cap = int(prob["stack_cap"])
        s.problem_id = problem_id
        if prob.get("nu_sigma_f") is not None:
            s.nu_sigma_f = _pd(arr(np.asarray(prob["nu_sigma_f"], float).reshape(M, G), np.float64))
            s.chi = _pd(arr(np.asarray(prob["chi"], float).reshape(M, G), np.float64))
        self.s = s
        mn = [int(v) for v in m["n"]]
        self.nbins = (G if m["per_group"] else 1) * mn[0] * mn[1] * mn[2] * mn[3]
        self.n_surf = 0
        if sf is not None:
            a = int(sf["axis"])
            b1, b2 = (1, 2) if a == 0 else ((0, 2) if a == 1 else (0, 1))
            self.n_surf = 2 * (G if m["per_group"] else 1) * mn[3] * mn[b1] * mn[b2]
        self.n_imp = G * int(np.prod(imp["n"])) if imp is not None else 0


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle returned status {status}")
        self.status = status


class OracleRun:
    """Accumulating oracle state for one problem (mirrors create/run/get)."""

    def __init__(self, prob: dict, problem_id: int = 0):
        self.prob = prob
        self.P = _Problem(prob, problem_id)
        nb = self.P.nbins
        self.tally_batch = np.zeros(nb)
        self.tally_sum = np.zeros(nb)
        self.tally_sumsq = np.zeros(nb)
        self.imp_score = np.zeros(max(self.P.n_imp, 1))
        self.imp_weight = np.zeros(max(self.P.n_imp, 1))
        self.R = OrcResult()
        self.R.tally_batch, self.R.tally_sum, self.R.tally_sumsq = (
            _pd(self.tally_batch), _pd(self.tally_sum), _pd(self.tally_sumsq))
        if prob.get("collision_tally"):
            self.col_batch = np.zeros(nb)
            self.col_sum = np.zeros(nb)
            self.col_sumsq = np.zeros(nb)
            self.R.col_batch, self.R.col_sum, self.R.col_sumsq = (
                _pd(self.col_batch), _pd(self.col_sum), _pd(self.col_sumsq))
        if self.P.n_surf:
            ns = self.P.n_surf
            self.surf_batch = np.zeros(ns)
            self.surf_sum = np.zeros(ns)
            self.surf_sumsq = np.zeros(ns)
            self.R.surf_batch, self.R.surf_sum, self.R.surf_sumsq = (
                _pd(self.surf_batch), _pd(self.surf_sum), _pd(self.surf_sumsq))
        if self.P.n_imp:
            self.R.imp_score, self.R.imp_weight = _pd(self.imp_score), _pd(self.imp_weight)
        self.n_hist = 0
        self.last_seconds = 0.0

    def run(self, n_hist: int, seed: int, trace_cap: int = 0, per_history: bool = False,
            first_id: int | None = None):
        """Transport ``n_hist`` histories with ids continuing from earlier runs.
        Returns (trace records, per-history [detector score, sum of w*d]) when
        asked."""
        trace = None
        xh = None
        if trace_cap:
            trace = np.zeros(trace_cap, TRACE_DTYPE)
            self.R.trace = trace.ctypes.data_as(C.POINTER(OrcTraceRec))
            self.R.trace_cap = trace_cap
            self.R.trace_n = 0
        else:
            self.R.trace = C.POINTER(OrcTraceRec)()
            self.R.trace_cap = 0
            self.R.trace_n = 0
        if per_history:
            xh = np.zeros((n_hist, 2))
            self.R.hist_xh = _pd(xh)
        else:
            self.R.hist_xh = PD()
        t0 = time.perf_counter()
        h0 = self.n_hist if first_id is None else int(first_id)
        st = lib().orc_run(C.byref(self.P.s), seed, h0, n_hist, C.byref(self.R))
        self.last_seconds = time.perf_counter() - t0
        if st != 0:
            raise OracleError(st)
        self.n_hist += n_hist
        if trace is not None:
            trace = trace[: self.R.trace_n].copy()
        return trace, xh

    def run_keff(self, M: int, n_inactive: int, n_active: int, seed: int, k0: float = 1.0,
                 trace_cap: int = 0, per_history: bool = False, src_out: bool = False):
        """k-eigenvalue power iteration (histories g M + j); tallies score in
        the active generations, one batch each.  Returns a dict with per
        generation k_col, k_site, n_sites, and optionally the trace, the
        per-history (detector score, path) of every generation and the last
        combed source [M][x, y, z, g]."""
        n_gen = n_inactive + n_active
        out = dict(k_col=np.zeros(n_gen), k_site=np.zeros(n_gen),
                   n_sites=np.zeros(n_gen, np.uint64))
        K = OrcKeff()
        K.M, K.n_inactive, K.n_active, K.k0 = M, n_inactive, n_active, k0
        K.k_col, K.k_site = _pd(out["k_col"]), _pd(out["k_site"])
        K.n_sites = out["n_sites"].ctypes.data_as(C.POINTER(C.c_uint64))
        src = np.zeros((M, 4)) if src_out else None
        K.src_out = _pd(src) if src_out else PD()
        trace = None
        if trace_cap:
            trace = np.zeros(trace_cap, TRACE_DTYPE)
            self.R.trace = trace.ctypes.data_as(C.POINTER(OrcTraceRec))
            self.R.trace_cap = trace_cap
        else:
            self.R.trace = C.POINTER(OrcTraceRec)()
            self.R.trace_cap = 0
        self.R.trace_n = 0
        xh = np.zeros((n_gen * M, 2)) if per_history else None
        self.R.hist_xh = _pd(xh) if per_history else PD()
        t0 = time.perf_counter()
        st = lib().orc_run_keff(C.byref(self.P.s), seed, C.byref(K), C.byref(self.R))
        self.last_seconds = time.perf_counter() - t0
        if st != 0:
            raise OracleError(st)
        self.n_hist += M * n_active
        if trace is not None:
            out["trace"] = trace[: self.R.trace_n].copy()
        if per_history:
            out["xh"] = xh
        if src_out:
            out["src"] = src
        return out

    @staticmethod
    def keff_stats(k_gen, n_inactive):
        """Mean of the active generations' estimates and its standard error
        (sample variance over n_active - 1, divided by n_active)."""
        k = np.asarray(k_gen, float)[n_inactive:]
        n = k.size
        m = float(np.mean(k))
        se = float(np.sqrt(np.sum((k - m) ** 2) / (n * (n - 1)))) if n > 1 else float("nan")
        return m, se

    # ---- results -------------------------------------------------------
    @property
    def counters(self) -> dict:
        return {k: int(self.R.cnt[i]) for i, k in enumerate(COUNTER_NAMES)}

    @property
    def wsum(self) -> dict:
        return {k: float(self.R.wsum[i]) for i, k in enumerate(WSUM_NAMES)}

    @property
    def leak(self) -> np.ndarray:
        return np.array(self.R.leak[:])

    @property
    def detector(self):
        """(sum x_h, sum x_h^2) over histories."""
        return float(self.R.det[0]), float(self.R.det[1])

    def mesh_stats(self, estimator: str = "track"):
        """Per-bin mean score per source particle and its standard error from
        batch means (weighted form for unequal batches); estimator "track"
        (track length), "collision", or "surface" (surface-current bins
        [side][group][t][b2][b1], side 0 crossing in +axis direction)."""
        N = float(self.n_hist)
        B = int(self.R.batches_done)
        s1, s2 = {"track": (self.tally_sum, self.tally_sumsq),
                  "collision": (getattr(self, "col_sum", None), getattr(self, "col_sumsq", None)),
                  "surface": (getattr(self, "surf_sum", None),
                              getattr(self, "surf_sumsq", None))}[estimator]
        mean = s1 / N
        if B < 2:
            return mean, np.full_like(mean, np.nan)
        var = (s2 - N * mean * mean) / ((B - 1) * N)
        return mean, np.sqrt(np.maximum(var, 0.0))

    def detector_stats(self):
        """Mean detector score per history and its standard error (the sample
        variance of the per-history scores over N - 1, divided by N)."""
        N = float(self.n_hist)
        s1, s2 = self.detector
        m = s1 / N
        if N < 2:
            return m, float("nan")
        var = (s2 / N - m * m) / (N - 1.0)
        return m, float(np.sqrt(max(var, 0.0)))

    def report(self, kind: str):
        """The run's output: tallies with their statistical error (the paper's
        problem statement and the finalization step of Sec. "MC/DC on CPUs").

        kind "mesh" / "collision": per bin, the mean score per source history
        divided by the bin's volume and time width (the space- and
        time-averaged flux); "surface": the mean crossing weight per source
        history divided by the bin's area on the plane and its time width;
        "detector": the mean track length per history in the detector box;
        "leakage": the weight leaked per face per history.  Returns (mean,
        rel) with rel = standard error / mean: 0 where the mean is 0, NaN with
        fewer than two batches (mesh kinds) or histories (detector), and NaN
        for leakage, which keeps no second moment."""
        N = float(self.n_hist)
        if kind == "detector":
            m, se = self.detector_stats()
            if np.isnan(se):
                return np.array([m]), np.array([np.nan])
            return np.array([m]), np.array([se / m if m > 0.0 else 0.0])
        if kind == "leakage":
            return self.leak / N, np.full(6, np.nan)
        est = {"mesh": "track", "collision": "collision", "surface": "surface"}[kind]
        mean, se = self.mesh_stats(est)
        msh = self.prob["mesh"]
        lo = np.asarray(msh["lo"], float)
        hi = np.asarray(msh["hi"], float)
        nn = np.asarray(msh["n"])
        skip = int(self.prob["surface_tally"]["axis"]) if kind == "surface" else -1
        size = 1.0
        for a in range(4):
            if a == skip or (a < 3 and np.isinf(lo[a]) and np.isinf(hi[a])):
                continue                      # an unbounded axis is not cut
            size *= (hi[a] - lo[a]) / float(nn[a])
        rel = np.where(mean > 0.0, se / np.where(mean > 0.0, mean, 1.0), 0.0)
        if int(self.R.batches_done) < 2:
            rel = np.full_like(mean, np.nan)
        return mean / size, rel


def run(prob: dict, n_hist: int, seed: int, **kw) -> OracleRun:
    r = OracleRun(prob)
    r.run(n_hist, seed, **kw)
    return r


# ---- primitives ------------------------------------------------------------

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def uniform(seed, hist, problem, tag, k):
    return lib().orc_uniform(seed, hist, problem, tag, k)


def log(x):
    return lib().orc_log(float(x))


def exp(x):
    return lib().orc_exp(float(x))


def directions(seed, hist, n):
    u = np.zeros((n, 3))
    k = lib().orc_directions(seed, hist, n, _pd(u))
    return u, int(k)


def mlp_f32(params, in_dim, hidden, x):
    p = np.ascontiguousarray(params, np.float32)
    xx = np.ascontiguousarray(x, np.float32)
    return float(lib().orc_mlp_f32(p.ctypes.data_as(PF), in_dim, hidden, xx.ctypes.data_as(PF)))


def score_segment(prob, p, u, t0, d, w=1.0, g=0):
    P = _Problem(prob)
    tally = np.zeros(P.nbins)
    pp = np.ascontiguousarray(p, float)
    uu = np.ascontiguousarray(u, float)
    n = lib().orc_score_segment(C.byref(P.s), _pd(pp), _pd(uu), t0, d, w, g, _pd(tally))
    return tally, int(n)


def ww_map(prob):
    """Weight-window map w_T[g][it][iz][iy][ix] of a problem whose ``ww`` has a ``map``."""
    P = _Problem(prob)
    n = [int(v) for v in prob["ww"]["map"]]
    out = np.zeros(P.s.G * n[0] * n[1] * n[2] * n[3])
    c = lib().orc_ww_map(C.byref(P.s), _pd(out))
    if c < 0:
        raise ValueError("problem has no weight-window map")
    return out.reshape(P.s.G, n[3], n[2], n[1], n[0])


def ww_map_cell(prob, p, t, g=0):
    """Flat map cell that the check uses for the point (p, t) in group g."""
    P = _Problem(prob)
    pp = np.ascontiguousarray(p, float)
    return int(lib().orc_ww_map_cell(C.byref(P.s), _pd(pp), float(t), int(g)))
