"""Python binding of libmcdc (ctypes).

Argument marshalling only: every step of the transport loop runs in the HIP
kernels of ``libmcdc.so``.  PyTorch provides device memory (the caller-owned
workspace and output buffers are torch tensors on ``cuda:0``) and the HIP
stream (``torch.cuda.current_stream().cuda_stream``).  If the library has not
been built, importing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# PyTorch first: its bundled HIP runtime and the one libmcdc.so links against
# share the soname libamdhip64.so.7, and the copy loaded first serves the whole
# process.  Loading torch's copy first keeps torch and the library on one
# runtime, the one torch was built with.
import torch  # noqa: F401  (import order matters)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcdc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2409_04668_amd.build` "
                      "(there is no CPU fallback)")

_lib = C.CDLL(LIB_PATH)

OK = 0
E_INVALID, E_NOMEM, E_HIP, E_EVENT_CAP, E_CANCELLED, E_STATE, E_STACK, E_BANK = -1, -2, -3, -4, -5, -6, -7, -8
E_EXTINCT = -9
SCHED_AUTO, SCHED_HISTORY, SCHED_EVENT, SCHED_HYBRID = 0, 1, 2, 3
TALLY_MESH, TALLY_DETECTOR, TALLY_LEAKAGE, TALLY_COLLISION, TALLY_SURFACE = 0, 1, 2, 3, 4
MAX_G = 8
HIDDEN = 64

D3 = C.c_double * 3
D4 = C.c_double * 4
I4 = C.c_int32 * 4
I6 = C.c_int32 * 6
PD = C.POINTER(C.c_double)
PI = C.POINTER(C.c_int32)
VP = C.c_void_p


class ProblemDesc(C.Structure):
    _fields_ = [
        ("outer_lo", D3), ("outer_hi", D3), ("bc", I6), ("n_boxes", C.c_int32),
        ("box_lo", PD), ("box_hi", PD), ("box_mat", PI), ("background_mat", C.c_int32),
        ("n_mat", C.c_int32), ("G", C.c_int32), ("sigma_t", PD), ("sigma_s", PD), ("speed", PD),
        ("src_kind", C.c_int32), ("src_lo", D3), ("src_hi", D3), ("src_t0", C.c_double),
        ("src_t1", C.c_double), ("src_isotropic", C.c_int32), ("src_dir", D3),
        ("src_group", C.c_int32), ("mesh_lo", D4), ("mesh_hi", D4), ("mesh_n", I4),
        ("mesh_per_group", C.c_int32), ("col_tally", C.c_int32), ("surf_on", C.c_int32),
        ("surf_axis", C.c_int32), ("surf_pos", C.c_double), ("pc_on", C.c_int32),
        ("pc_target", C.c_double),
        ("n_census", C.c_int32), ("census", PD),
        ("implicit_capture", C.c_int32), ("w_cut", C.c_double), ("w_surv", C.c_double),
        ("has_detector", C.c_int32), ("det_lo", D3), ("det_hi", D3), ("imp_on", C.c_int32),
        ("imp_n", I4), ("n_batches", C.c_int32), ("max_events", C.c_int64),
        ("stack_cap", C.c_int32), ("problem_id", C.c_uint32),
        ("nu_sigma_f", PD), ("chi", PD),
    ]


class KeffOpts(C.Structure):
    _fields_ = [("M", C.c_uint64), ("n_inactive", C.c_int32), ("n_active", C.c_int32),
                ("k0", C.c_double)]


class Options(C.Structure):
    _fields_ = [("schedule", C.c_int32), ("block", C.c_int32), ("waves_per_cu", C.c_int32),
                ("lds_tally", C.c_int32), ("event_chunk", C.c_int64),
                ("tile_lo", C.c_int32 * 5), ("tile_n", C.c_int32 * 5)]


MAX_TILE_BINS = 19456


COUNTER_FIELDS = ["histories", "flights", "pieces", "collisions", "absorptions", "surfaces",
                  "leaks", "census_stops", "time_ends", "splits", "rr_kills", "rr_survivals",
                  "cutoff_kills", "cutoff_survivals", "detector_hits", "particles"]


class RunState(C.Structure):
    _fields_ = [("magic", C.c_uint64), ("workspace_bytes", C.c_uint64), ("bins", C.c_uint64),
                ("n_hist", C.c_uint64), ("batches", C.c_uint64), ("event_iterations", C.c_uint64),
                ("run_first", C.c_uint64), ("run_n", C.c_uint64), ("run_seed", C.c_uint64),
                ("segment", C.c_uint64), ("in_run", C.c_int32), ("steps", C.c_int32)]


class Counters(C.Structure):
    _fields_ = ([(n, C.c_uint64) for n in COUNTER_FIELDS] +
                [(n, C.c_double) for n in ["w_source", "w_leak", "w_absorb", "w_time_end",
                                           "w_gain", "w_loss", "path"]] +
                [("leak", C.c_double * 6), ("det_sum", C.c_double), ("det_sumsq", C.c_double),
                 ("batches", C.c_int64), ("n_hist", C.c_uint64), ("status", C.c_int32),
                 ("event_iterations", C.c_uint64), ("pc_kills", C.c_uint64),
                 ("pc_copies", C.c_uint64), ("surf_crossings", C.c_uint64),
                 ("ww_plane_stops", C.c_uint64)])

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n != "leak"}
        d["leak"] = np.array(self.leak[:])
        return d


TRACE_DTYPE = np.dtype([("hist", "<u8"), ("tag", "<u4"), ("seq", "<u4"), ("type", "<i4"),
                        ("g", "<i4"), ("cell", "<i4"), ("k", "<u4"), ("x", "<f8"), ("y", "<f8"),
                        ("z", "<f8"), ("t", "<f8"), ("ux", "<f8"), ("uy", "<f8"), ("uz", "<f8"),
                        ("w", "<f8"), ("aux", "<f8")])


class TrainOpts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("mcdc_workspace_bytes", C.c_int, C.POINTER(ProblemDesc), C.POINTER(Options), C.POINTER(C.c_size_t))
_sig("mcdc_create_problem", C.c_int, C.POINTER(ProblemDesc), C.POINTER(Options), VP, C.c_size_t,
     C.POINTER(VP))
_sig("mcdc_run", C.c_int, VP, C.c_uint64, C.c_uint64, VP)
_sig("mcdc_run_begin", C.c_int, VP, C.c_uint64, C.c_uint64, VP)
_sig("mcdc_run_step", C.c_int, VP, C.POINTER(C.c_int32), VP)
_sig("mcdc_get_run_state", C.c_int, VP, VP)
_sig("mcdc_set_run_state", C.c_int, VP, VP)
_sig("mcdc_get_tallies", C.c_int, VP, C.c_int, PD, PD, C.c_size_t, VP)
_sig("mcdc_get_tallies_device", C.c_int, VP, C.c_int, VP, VP, C.c_size_t, VP)
_sig("mcdc_set_cancel", C.c_int, VP, C.c_int)
_sig("mcdc_keff_workspace_bytes", C.c_int, C.c_uint64, C.POINTER(C.c_size_t))
_sig("mcdc_run_keff", C.c_int, VP, C.POINTER(KeffOpts), C.c_uint64, VP, C.c_size_t, PD, PD,
     C.POINTER(C.c_uint64), VP)
_sig("mcdc_get_raw", C.c_int, VP, PD, PD, C.c_size_t, VP)
_sig("mcdc_get_raw_collision", C.c_int, VP, PD, PD, C.c_size_t, VP)
_sig("mcdc_get_raw_surface", C.c_int, VP, PD, PD, C.c_size_t, VP)
_sig("mcdc_surface_bins", C.c_int, VP, C.POINTER(C.c_size_t))
_sig("mcdc_get_counters", C.c_int, VP, C.POINTER(Counters), VP)
_sig("mcdc_reset_tallies", C.c_int, VP, VP)
_sig("mcdc_tally_bins", C.c_int, VP, C.POINTER(C.c_size_t))
_sig("mcdc_set_trace", C.c_int, VP, VP, C.c_uint64, VP)
_sig("mcdc_set_history_scores", C.c_int, VP, VP)
_sig("mcdc_set_ww_mlp", C.c_int, VP, C.POINTER(C.c_float), C.c_size_t, C.c_double, C.c_double,
     C.c_int32, C.c_float, C.c_float)
_sig("mcdc_set_ww_map", C.c_int, VP, C.POINTER(C.c_int32), VP, C.c_size_t, VP)
_sig("mcdc_set_ww_grid", C.c_int, VP, C.POINTER(C.c_int32))
_sig("mcdc_get_importance", C.c_int, VP, PD, PD, C.c_size_t, VP)
_sig("mcdc_mlp_param_count", C.c_size_t, C.c_int32)
_sig("mcdc_mlp_forward", C.c_int, VP, C.c_int32, VP, C.c_size_t, VP, VP)
_sig("mcdc_mlp_scratch_bytes", C.c_size_t, C.c_int32, C.c_size_t)
_sig("mcdc_mlp_grad", C.c_int, VP, C.c_int32, VP, VP, VP, C.c_size_t, VP, VP, VP, VP)
_sig("mcdc_mlp_train", C.c_int, VP, C.c_int32, VP, VP, VP, C.c_size_t, VP, VP, VP,
     C.POINTER(TrainOpts), C.POINTER(C.c_int32), VP, VP, VP)
_sig("mcdc_mlp_train_noalloc", C.c_int, VP, C.c_int32, VP, VP, VP, C.c_size_t, VP, VP, VP,
     C.POINTER(TrainOpts), C.POINTER(C.c_int32), VP, VP)
_sig("mcdc_batch_workspace_bytes", C.c_int, C.POINTER(ProblemDesc), C.c_size_t,
     C.POINTER(C.c_uint64), C.POINTER(Options), C.POINTER(C.c_size_t))
_sig("mcdc_create_batch", C.c_int, C.POINTER(ProblemDesc), C.c_size_t, C.POINTER(C.c_uint64),
     C.POINTER(Options), VP, C.c_size_t, C.POINTER(VP))
_sig("mcdc_run_batch", C.c_int, VP, C.c_uint64, VP)
_sig("mcdc_get_batch_raw", C.c_int, VP, C.c_size_t, PD, C.c_size_t, VP)
_sig("mcdc_get_batch_counters", C.c_int, VP, C.c_size_t, C.POINTER(Counters), VP)
_sig("mcdc_get_batch_history_path", C.c_int, VP, C.c_size_t, PD, C.c_size_t, VP)
_sig("mcdc_micro_atomics", C.c_int, VP, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, VP)
_sig("mcdc_micro_lds_atomics", C.c_int, VP, C.c_uint32, C.c_uint64, C.c_uint32, VP)
_sig("mcdc_micro_copy", C.c_int, VP, VP, C.c_size_t, VP)
_sig("mcdc_set_kernel_timing", C.c_int, VP, C.c_int)
_sig("mcdc_kernel_time", C.c_int, VP, C.POINTER(C.c_uint64), C.POINTER(C.c_double))
_sig("mcdc_destroy_problem", None, VP)
_sig("mcdc_last_error", C.c_char_p)


class McdcError(RuntimeError):
    def __init__(self, status, where):
        msg = _lib.mcdc_last_error().decode(errors="replace")
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def check(st, where):
    if st != OK:
        raise McdcError(st, where)


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return VP(s.cuda_stream)


def _ptr(t):
    return VP(t.data_ptr())


class _Desc:
    """ProblemDesc plus the host arrays it points to."""

    def __init__(self, prob: dict, problem_id: int = 0):
        self.keep = []

        def arr(x, dt):
            a = np.ascontiguousarray(np.asarray(x, dtype=dt))
            self.keep.append(a)
            return a

        d = ProblemDesc()
        d.outer_lo = D3(*map(float, prob["outer_lo"]))
        d.outer_hi = D3(*map(float, prob["outer_hi"]))
        d.bc = I6(*map(int, prob["bc"]))
        nb = int(np.asarray(prob["box_mat"]).size)
        d.n_boxes = nb
        blo = arr(np.asarray(prob["box_lo"], float).reshape(-1, 3) if nb else np.zeros((1, 3)), np.float64)
        bhi = arr(np.asarray(prob["box_hi"], float).reshape(-1, 3) if nb else np.zeros((1, 3)), np.float64)
        bm = arr(prob["box_mat"] if nb else np.zeros(1), np.int32)
        d.box_lo = blo.ctypes.data_as(PD)
        d.box_hi = bhi.ctypes.data_as(PD)
        d.box_mat = bm.ctypes.data_as(PI)
        d.background_mat = int(prob["background_mat"])
        st = arr(prob["sigma_t"], np.float64)
        M, G = st.shape
        d.n_mat, d.G = M, G
        ss = arr(np.asarray(prob["sigma_s"], float).reshape(M, G, G), np.float64)
        sp = arr(prob["speed"], np.float64)
        d.sigma_t, d.sigma_s, d.speed = st.ctypes.data_as(PD), ss.ctypes.data_as(PD), sp.ctypes.data_as(PD)
        src = prob["source"]
        d.src_kind = 1 if src["kind"] == "box" else 0
        d.src_lo = D3(*map(float, src["lo"]))
        d.src_hi = D3(*map(float, src["hi"]))
        d.src_t0, d.src_t1 = float(src["t0"]), float(src["t1"])
        d.src_isotropic = 1 if src["isotropic"] else 0
        d.src_dir = D3(*map(float, src["dir"]))
        d.src_group = int(src["group"])
        m = prob["mesh"]
        d.mesh_lo = D4(*map(float, m["lo"]))
        d.mesh_hi = D4(*map(float, m["hi"]))
        d.mesh_n = I4(*map(int, m["n"]))
        d.mesh_per_group = 1 if m["per_group"] else 0
        d.col_tally = 1 if prob.get("collision_tally") else 0
        sf = prob.get("surface_tally")
        d.surf_on = 1 if sf is not None else 0
        if sf is not None:
            d.surf_axis = int(sf["axis"])
            d.surf_pos = float(sf["pos"])
        pc = prob.get("population_control")
        d.pc_on = 1 if pc is not None else 0
        d.pc_target = float(pc["target"]) if pc is not None else 0.0
        cen = arr(prob["census"], np.float64)
        d.n_census, d.census = cen.size, cen.ctypes.data_as(PD)
        d.implicit_capture = 1 if prob["implicit_capture"] else 0
        d.w_cut, d.w_surv = float(prob["w_cut"]), float(prob["w_surv"])
        det = prob.get("detector")
        d.has_detector = 1 if det is not None else 0
        if det is not None:
            d.det_lo = D3(*map(float, det["lo"]))
            d.det_hi = D3(*map(float, det["hi"]))
        imp = prob.get("importance")
        d.imp_on = 1 if imp is not None else 0
        if imp is not None:
            d.imp_n = I4(*map(int, imp["n"]))
        d.n_batches = int(prob["n_batches"])
        d.max_events = int(prob["max_events"])
        # daughter stack storage is only carved when weight windows may be used
        d.stack_cap = int(prob["stack_cap"]) if prob.get("ww") is not None else 0
        d.problem_id = problem_id
        if prob.get("nu_sigma_f") is not None:
            d.nu_sigma_f = arr(np.asarray(prob["nu_sigma_f"], float).reshape(M, G), np.float64).ctypes.data_as(PD)
            d.chi = arr(np.asarray(prob["chi"], float).reshape(M, G), np.float64).ctypes.data_as(PD)
        self.d = d
        self.G = G
        mn = [int(v) for v in m["n"]]
        self.nbins = (G if m["per_group"] else 1) * mn[0] * mn[1] * mn[2] * mn[3]
        self.nimp = G * int(np.prod(imp["n"])) if imp is not None else 0


def make_options(schedule=SCHED_HISTORY, block=0, waves_per_cu=0, lds_tally=1, event_chunk=0,
                 tile=None):
    """tile = (lo[5], n[5]) in bins along x, y, z, t, group: LDS hot tile."""
    o = Options()
    o.schedule, o.block, o.waves_per_cu, o.lds_tally, o.event_chunk = (
        schedule, block, waves_per_cu, lds_tally, event_chunk)
    if tile is not None:
        lo, n = tile
        o.tile_lo = (C.c_int32 * 5)(*[int(v) for v in lo])
        o.tile_n = (C.c_int32 * 5)(*[int(v) for v in n])
    return o


class Problem:
    """One problem on the GPU: workspace tensor + library handle."""

    def __init__(self, prob: dict, options: Options | None = None, device="cuda:0",
                 problem_id: int = 0):
        import torch
        self.torch = torch
        self.prob = prob
        self.desc = _Desc(prob, problem_id)
        self.opt = options if options is not None else make_options()
        nbytes = C.c_size_t()
        check(_lib.mcdc_workspace_bytes(C.byref(self.desc.d), C.byref(self.opt), C.byref(nbytes)),
              "workspace_bytes")
        self.ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=device)
        h = VP()
        check(_lib.mcdc_create_problem(C.byref(self.desc.d), C.byref(self.opt), _ptr(self.ws),
                                       nbytes.value, C.byref(h)), "create_problem")
        self.h = h
        self.nbins = self.desc.nbins
        self._trace = None
        self._xh = None
        self._ww_map = None
        ww = prob.get("ww")
        if ww is not None:
            self.set_ww(ww["params"], ww["logk"], ww.get("ratio", 5.0), ww.get("n_max", 10),
                        ww.get("ymin", -3.0e38), ww.get("ymax", 3.0e38))
            if ww.get("map") is not None:
                self.set_ww_map(ww["map"])
            if ww.get("grid") is not None:
                self.set_ww_grid(ww["grid"])

    def close(self):
        if self.h:
            _lib.mcdc_destroy_problem(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- running -------------------------------------------------------
    def run(self, n_hist: int, seed: int, stream=None):
        check(_lib.mcdc_run(self.h, int(n_hist), int(seed), _stream_ptr(stream)), "run")

    def run_keff(self, M: int, n_inactive: int, n_active: int, seed: int, k0: float = 1.0,
                 stream=None) -> dict:
        """k-eigenvalue power iteration (histories g M + j); returns per
        generation k_col, k_site and n_sites.  The site banks live in a
        device tensor held for the call."""
        t = self.torch
        nbytes = C.c_size_t()
        check(_lib.mcdc_keff_workspace_bytes(int(M), C.byref(nbytes)), "keff_workspace_bytes")
        ws = t.empty(int(nbytes.value), dtype=t.uint8, device=self.ws.device)
        n_gen = int(n_inactive) + int(n_active)
        out = dict(k_col=np.zeros(max(n_gen, 1)), k_site=np.zeros(max(n_gen, 1)),
                   n_sites=np.zeros(max(n_gen, 1), np.uint64))
        o = KeffOpts(int(M), int(n_inactive), int(n_active), float(k0))
        st = _lib.mcdc_run_keff(self.h, C.byref(o), int(seed), _ptr(ws), nbytes.value,
                                out["k_col"].ctypes.data_as(PD), out["k_site"].ctypes.data_as(PD),
                                out["n_sites"].ctypes.data_as(C.POINTER(C.c_uint64)),
                                _stream_ptr(stream))
        del ws
        check(st, "run_keff")
        return {k: v[:n_gen] for k, v in out.items()}

    # ---- stepped runs: census step by census step, segment by segment --
    def run_begin(self, n_hist: int, seed: int, stream=None):
        check(_lib.mcdc_run_begin(self.h, int(n_hist), int(seed), _stream_ptr(stream)), "run_begin")

    def run_step(self, stream=None) -> bool:
        """Transport to the next census step or segment; True when the run has ended."""
        done = C.c_int32(0)
        check(_lib.mcdc_run_step(self.h, C.byref(done), _stream_ptr(stream)), "run_step")
        return bool(done.value)

    def run_state(self) -> "RunState":
        st = RunState()
        check(_lib.mcdc_get_run_state(self.h, C.byref(st)), "get_run_state")
        return st

    def set_run_state(self, st: "RunState"):
        check(_lib.mcdc_set_run_state(self.h, C.byref(st)), "set_run_state")

    def set_trace(self, cap: int):
        """Record every event of later runs (device buffer of ``cap`` records)."""
        t = self.torch
        if cap:
            buf = t.zeros(cap * TRACE_DTYPE.itemsize, dtype=t.uint8, device=self.ws.device)
            cnt = t.zeros(1, dtype=t.int64, device=self.ws.device)
            check(_lib.mcdc_set_trace(self.h, _ptr(buf), cap, _ptr(cnt)), "set_trace")
            self._trace = (buf, cnt, cap)
        else:
            check(_lib.mcdc_set_trace(self.h, None, 0, None), "set_trace")
            self._trace = None

    def trace(self):
        buf, cnt, cap = self._trace
        self.torch.cuda.synchronize()
        n = min(int(cnt.item()), cap)
        return np.frombuffer(buf.cpu().numpy().tobytes(), dtype=TRACE_DTYPE)[:n].copy()

    def set_history_scores(self, n_hist: int | None):
        t = self.torch
        if n_hist:
            self._xh = t.zeros(2 * n_hist, dtype=t.float64, device=self.ws.device)
            check(_lib.mcdc_set_history_scores(self.h, _ptr(self._xh)), "set_history_scores")
        else:
            check(_lib.mcdc_set_history_scores(self.h, None), "set_history_scores")
            self._xh = None

    def history_scores(self):
        self.torch.cuda.synchronize()
        return self._xh.cpu().numpy().reshape(-1, 2)

    def set_ww(self, params, logk, ratio=5.0, n_max=10, ymin=-3.0e38, ymax=3.0e38):
        self._ww_map = None                     # a new network drops the baked map
        if params is None:
            check(_lib.mcdc_set_ww_mlp(self.h, None, 0, 0.0, 0.0, 0, 0.0, 0.0), "set_ww_mlp")
            return
        p = np.ascontiguousarray(params, np.float32)
        check(_lib.mcdc_set_ww_mlp(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size,
                                   float(logk), float(ratio), int(n_max), float(ymin), float(ymax)),
              "set_ww_mlp")

    def set_ww_map(self, dims, stream=None):
        """Bake the network onto a (nx, ny, nz, nt) cell-centre window map
        (device tensor owned here); ``dims=None`` returns to per-check inference."""
        if dims is None:
            check(_lib.mcdc_set_ww_map(self.h, None, None, 0, None), "set_ww_map")
            self._ww_map = None
            return
        n = (C.c_int32 * 4)(*[int(v) for v in dims])
        cells = self.desc.d.G * int(np.prod([int(v) for v in dims]))
        buf = self.torch.empty(max(cells, 1), dtype=self.torch.float64, device=self.ws.device)
        check(_lib.mcdc_set_ww_map(self.h, n, _ptr(buf), cells, _stream_ptr(stream)),
              "set_ww_map")
        self._ww_map = buf

    def set_ww_grid(self, n):
        """Window checks also on the interior planes of an n[0] x n[1] x n[2]
        grid over the outer box (None turns them off)."""
        if n is None:
            check(_lib.mcdc_set_ww_grid(self.h, None), "set_ww_grid")
            return
        arr = (C.c_int32 * 3)(*[int(v) for v in n])
        check(_lib.mcdc_set_ww_grid(self.h, arr), "set_ww_grid")

    def ww_map(self):
        """The baked window targets w_T as a host array [g][t][z][y][x]."""
        self.torch.cuda.synchronize()
        return self._ww_map.cpu().numpy()

    # ---- results -------------------------------------------------------
    def raw(self, stream=None):
        s = np.zeros(self.nbins)
        s2 = np.zeros(self.nbins)
        check(_lib.mcdc_get_raw(self.h, s.ctypes.data_as(PD), s2.ctypes.data_as(PD), self.nbins,
                                _stream_ptr(stream)), "get_raw")
        return s, s2

    def raw_collision(self, stream=None):
        s = np.zeros(self.nbins)
        s2 = np.zeros(self.nbins)
        check(_lib.mcdc_get_raw_collision(self.h, s.ctypes.data_as(PD), s2.ctypes.data_as(PD),
                                          self.nbins, _stream_ptr(stream)), "get_raw_collision")
        return s, s2

    def surface_bins(self) -> int:
        n = C.c_size_t()
        check(_lib.mcdc_surface_bins(self.h, C.byref(n)), "surface_bins")
        return int(n.value)

    def raw_surface(self, stream=None):
        """Surface-current sums [side][g][t][b2][b1] (side 0: crossing toward
        +axis) and batch sums of squares."""
        n = self.surface_bins()
        s = np.zeros(n)
        s2 = np.zeros(n)
        check(_lib.mcdc_get_raw_surface(self.h, s.ctypes.data_as(PD), s2.ctypes.data_as(PD), n,
                                        _stream_ptr(stream)), "get_raw_surface")
        return s, s2

    def tallies(self, kind=TALLY_MESH, stream=None):
        n = {TALLY_MESH: self.nbins, TALLY_DETECTOR: 1, TALLY_LEAKAGE: 6,
             TALLY_COLLISION: self.nbins}[kind] if kind != TALLY_SURFACE else self.surface_bins()
        m = np.zeros(n)
        r = np.zeros(n)
        check(_lib.mcdc_get_tallies(self.h, kind, m.ctypes.data_as(PD), r.ctypes.data_as(PD), n,
                                    _stream_ptr(stream)), "get_tallies")
        return m, r

    def tallies_device(self, kind=TALLY_MESH, stream=None, with_rel=True):
        """The same results as ``tallies`` computed into device tensors on the
        stream (no synchronisation)."""
        t = self.torch
        n = {TALLY_MESH: self.nbins, TALLY_DETECTOR: 1, TALLY_LEAKAGE: 6,
             TALLY_COLLISION: self.nbins}[kind] if kind != TALLY_SURFACE else self.surface_bins()
        # at least one element each, so that an empty result still passes a
        # non-null pointer (the library then reports the real problem)
        m = t.empty(max(n, 1), dtype=t.float64, device=self.ws.device)
        r = t.empty(max(n, 1), dtype=t.float64, device=self.ws.device) if with_rel else None
        check(_lib.mcdc_get_tallies_device(self.h, kind, _ptr(m), _ptr(r) if r is not None else None,
                                           n, _stream_ptr(stream)), "get_tallies_device")
        return m[:n], (r[:n] if r is not None else None)

    def set_cancel(self, on: bool = True):
        """Ask running and later runs to stop (thread safe); False clears it."""
        check(_lib.mcdc_set_cancel(self.h, 1 if on else 0), "set_cancel")

    def counters(self, stream=None) -> dict:
        c = Counters()
        check(_lib.mcdc_get_counters(self.h, C.byref(c), _stream_ptr(stream)), "get_counters")
        return c.as_dict()

    def importance(self, stream=None):
        n = self.desc.nimp
        s = np.zeros(n)
        w = np.zeros(n)
        check(_lib.mcdc_get_importance(self.h, s.ctypes.data_as(PD), w.ctypes.data_as(PD), n,
                                       _stream_ptr(stream)), "get_importance")
        return s, w

    def set_kernel_timing(self, on: bool):
        check(_lib.mcdc_set_kernel_timing(self.h, 1 if on else 0), "set_kernel_timing")

    def kernel_time(self):
        """(launches, total ms) of the tracking kernels since the last call."""
        n = C.c_uint64()
        ms = C.c_double()
        check(_lib.mcdc_kernel_time(self.h, C.byref(n), C.byref(ms)), "kernel_time")
        return int(n.value), float(ms.value)

    def reset(self, stream=None):
        check(_lib.mcdc_reset_tallies(self.h, _stream_ptr(stream)), "reset_tallies")


class BatchProblem:
    """Many independent problems run together: one persistent launch per census
    step, the census steps of a pass replayed from a HIP graph."""

    def __init__(self, probs, n_hist, options: Options | None = None, device="cuda:0"):
        import torch
        self.torch = torch
        self.probs = probs
        self.n_hist = np.ascontiguousarray(n_hist, np.uint64)
        self.descs = [_Desc(p, problem_id=i) for i, p in enumerate(probs)]
        arr = (ProblemDesc * len(probs))(*[d.d for d in self.descs])
        self._arr = arr
        self.opt = options if options is not None else make_options()
        nh = self.n_hist.ctypes.data_as(C.POINTER(C.c_uint64))
        nbytes = C.c_size_t()
        check(_lib.mcdc_batch_workspace_bytes(arr, len(probs), nh, C.byref(self.opt),
                                              C.byref(nbytes)), "batch_workspace_bytes")
        self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
        h = VP()
        check(_lib.mcdc_create_batch(arr, len(probs), nh, C.byref(self.opt), _ptr(self.ws),
                                     nbytes.value, C.byref(h)), "create_batch")
        self.h = h

    def close(self):
        if self.h:
            _lib.mcdc_destroy_problem(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, seed: int, stream=None):
        check(_lib.mcdc_run_batch(self.h, int(seed), _stream_ptr(stream)), "run_batch")

    def set_cancel(self, on: bool = True):
        check(_lib.mcdc_set_cancel(self.h, 1 if on else 0), "set_cancel")

    def raw(self, p: int, stream=None):
        n = self.descs[p].nbins
        s = np.zeros(n)
        check(_lib.mcdc_get_batch_raw(self.h, p, s.ctypes.data_as(PD), n, _stream_ptr(stream)),
              "get_batch_raw")
        return s

    def counters(self, p: int, stream=None) -> dict:
        c = Counters()
        check(_lib.mcdc_get_batch_counters(self.h, p, C.byref(c), _stream_ptr(stream)),
              "get_batch_counters")
        return c.as_dict()

    def history_path(self, p: int, stream=None):
        n = int(self.n_hist[p])
        out = np.zeros(n)
        check(_lib.mcdc_get_batch_history_path(self.h, p, out.ctypes.data_as(PD), n,
                                               _stream_ptr(stream)), "get_batch_history_path")
        return out


def micro_atomic_rate(n_bins: int, n_updates: int, run: int = 1, per_item: int = 64, reps: int = 3):
    """Measured FP64 atomic-add rate (updates/s) into an n_bins array."""
    import torch
    buf = torch.zeros(n_bins, dtype=torch.float64, device="cuda")
    n_items = max(1, n_updates // per_item)
    best = 0.0
    for _ in range(reps + 1):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        check(_lib.mcdc_micro_atomics(_ptr(buf), n_bins, n_items, per_item, run, _stream_ptr()),
              "micro_atomics")
        b.record()
        b.synchronize()
        best = max(best, n_items * per_item / (a.elapsed_time(b) / 1e3))
    total = float(buf.sum().item())
    assert total == float(n_items * per_item * (reps + 1)), "atomic micro-benchmark lost updates"
    return best


def micro_lds_atomic_rate(n_bins: int, n_updates: int, reps: int = 3):
    """Measured LDS FP64 atomic-add rate (ds_add_f64 updates/s) into an
    n_bins array per 1024-work-item workgroup, one workgroup per compute unit
    (zeroing and the final per-workgroup total included in the timed
    launch)."""
    import torch
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    n_items = torch.cuda.get_device_properties(0).multi_processor_count * 1024
    per_item = max(1, n_updates // n_items)
    best = 0.0
    for _ in range(reps + 1):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        check(_lib.mcdc_micro_lds_atomics(_ptr(out), n_bins, n_items, per_item, _stream_ptr()),
              "micro_lds_atomics")
        b.record()
        b.synchronize()
        best = max(best, n_items * per_item / (a.elapsed_time(b) / 1e3))
    total = float(out.sum().item())
    assert total == float(n_items * per_item * (reps + 1)), "LDS atomic micro-benchmark lost updates"
    return best


def micro_copy_rate(n_bytes: int = 1 << 30, reps: int = 3):
    """Measured device-to-device streaming rate (bytes moved / s, read + write)."""
    import torch
    n = n_bytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    best = 0.0
    for _ in range(reps + 1):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        check(_lib.mcdc_micro_copy(_ptr(src), _ptr(dst), n * 8, _stream_ptr()), "micro_copy")
        b.record()
        b.synchronize()
        best = max(best, 2 * n * 8 / (a.elapsed_time(b) / 1e3))
    return best


def mlp_param_count(in_dim: int) -> int:
    return int(_lib.mcdc_mlp_param_count(in_dim))


def exported_symbols():
    """Names of the C entry points this binding resolves."""
    return [n for n in dir(_lib) if n.startswith("mcdc_")]
