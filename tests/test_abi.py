"""The C-ABI library loads on the CPU and exports every entry point that
include/mcdc.h declares (no compute calls: those need a GPU)."""
import ctypes
import os
import re

import pytest
import torch  # noqa: F401  (load torch's HIP runtime before the library; same soname)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcdc.h")
LIB = os.path.join(ROOT, "paper_2409_04668_amd", "libmcdc.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mcdc_[a-z_0-9]+)\s*\(", src)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcdc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcdc.so not built")
def test_binding_imports_and_validates_on_cpu():
    import numpy as np
    from paper_2409_04668_amd import mcdc, workloads as W
    d = mcdc._Desc(W.config2())
    n = ctypes.c_size_t()
    assert mcdc._lib.mcdc_workspace_bytes(ctypes.byref(d.d), ctypes.byref(mcdc.make_options()),
                                          ctypes.byref(n)) == 0
    assert n.value >= 3 * 8 * W.n_bins(W.config2())
    p = W.config1()
    p["census"] = np.array([5.0, 4.0])
    bad = mcdc._Desc(p)
    st = mcdc._lib.mcdc_workspace_bytes(ctypes.byref(bad.d), ctypes.byref(mcdc.make_options()),
                                        ctypes.byref(n))
    assert st == mcdc.E_INVALID
    assert b"census" in mcdc._lib.mcdc_last_error()
    assert mcdc.mlp_param_count(5) == 4609


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcdc.so not built")
def test_failure_paths_without_gpu():
    """Errors are reported as status codes with a message before any device
    work: workspace too small, bad options, bad tiles, bad batches."""
    import numpy as np
    from paper_2409_04668_amd import mcdc, workloads as W
    d = mcdc._Desc(W.config2())
    n = ctypes.c_size_t()
    opt = mcdc.make_options()
    assert mcdc._lib.mcdc_workspace_bytes(ctypes.byref(d.d), ctypes.byref(opt), ctypes.byref(n)) == 0
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)            # never dereferenced: the size check fails first
    st = mcdc._lib.mcdc_create_problem(ctypes.byref(d.d), ctypes.byref(opt), fake, n.value - 256,
                                       ctypes.byref(h))
    assert st == mcdc.E_NOMEM and b"too small" in mcdc._lib.mcdc_last_error()
    bad = mcdc.make_options(block=100)
    assert mcdc._lib.mcdc_workspace_bytes(ctypes.byref(d.d), ctypes.byref(bad),
                                          ctypes.byref(n)) == mcdc.E_INVALID
    big = mcdc.make_options(tile=([0, 0, 0, 0, 0], [60, 100, 60, 20, 1]))
    assert mcdc._lib.mcdc_workspace_bytes(ctypes.byref(d.d), ctypes.byref(big),
                                          ctypes.byref(n)) == mcdc.E_INVALID
    p = W.config2()
    p["box_mat"] = np.array([0, 1, 7, 1], np.int32)          # material out of range
    bd = mcdc._Desc(p)
    assert mcdc._lib.mcdc_workspace_bytes(ctypes.byref(bd.d), ctypes.byref(opt),
                                          ctypes.byref(n)) == mcdc.E_INVALID
    # batched problems must share their census count
    probs = [W.batch_problem(1), W.batch_problem(2, nt=5)]
    descs = [mcdc._Desc(q, i) for i, q in enumerate(probs)]
    arr = (mcdc.ProblemDesc * 2)(*[x.d for x in descs])
    nh = (ctypes.c_uint64 * 2)(10, 10)
    st = mcdc._lib.mcdc_batch_workspace_bytes(arr, 2, nh, ctypes.byref(opt), ctypes.byref(n))
    assert st == mcdc.E_INVALID and b"census" in mcdc._lib.mcdc_last_error()
    # the weight-window map needs a handle
    dims = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    assert mcdc._lib.mcdc_set_ww_map(None, dims, None, 0, None) == mcdc.E_INVALID
    # census-step control needs a handle
    done = ctypes.c_int32()
    assert mcdc._lib.mcdc_run_step(None, ctypes.byref(done), None) == mcdc.E_INVALID
    st = mcdc.RunState()
    assert mcdc._lib.mcdc_get_run_state(None, ctypes.byref(st)) == mcdc.E_INVALID
    # k-eigenvalue sizing and arguments
    assert mcdc._lib.mcdc_keff_workspace_bytes(0, ctypes.byref(n)) == mcdc.E_INVALID
    assert mcdc._lib.mcdc_keff_workspace_bytes(1 << 29, ctypes.byref(n)) == mcdc.E_INVALID
    assert mcdc._lib.mcdc_keff_workspace_bytes(1000, ctypes.byref(n)) == 0
    assert n.value >= (3 + 3) * 8 * (4 * 1000 + 1024)         # unordered and ordered site banks
    ko = mcdc.KeffOpts(1000, 0, 1, 1.0)
    assert mcdc._lib.mcdc_run_keff(None, ctypes.byref(ko), 1, None, 0, None, None, None,
                                   None) == mcdc.E_INVALID
    assert mcdc._lib.mcdc_set_cancel(None, 1) == mcdc.E_INVALID
    # fission data: a spectrum is required, and must be non-negative
    p = W.keff_infinite_medium([1.0], [[0.6]], [0.5], [1.0])
    p["chi"] = np.array([[-1.0]])
    bad = mcdc._Desc(p)
    assert mcdc._lib.mcdc_workspace_bytes(ctypes.byref(bad.d), ctypes.byref(opt),
                                          ctypes.byref(n)) == mcdc.E_INVALID
    p["chi"] = np.array([[0.0]])
    bad = mcdc._Desc(p)
    assert mcdc._lib.mcdc_workspace_bytes(ctypes.byref(bad.d), ctypes.byref(opt),
                                          ctypes.byref(n)) == mcdc.E_INVALID
    # fissile problems do not batch
    q = W.batch_problem(3)
    q["nu_sigma_f"] = np.full(q["sigma_t"].shape, 0.1)
    q["chi"] = np.ones(q["sigma_t"].shape)
    dq = mcdc._Desc(q)
    arr1 = (mcdc.ProblemDesc * 1)(dq.d)
    nh1 = (ctypes.c_uint64 * 1)(10)
    assert mcdc._lib.mcdc_batch_workspace_bytes(arr1, 1, nh1, ctypes.byref(opt),
                                                ctypes.byref(n)) == mcdc.E_INVALID


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcdc.so not built")
def test_surface_tally_description_is_validated_on_cpu():
    import numpy as np
    from paper_2409_04668_amd import mcdc, workloads as W
    n = ctypes.c_size_t()
    p = W.config2()
    p["surface_tally"] = dict(axis=1, pos=40.0)
    d = mcdc._Desc(p)
    assert mcdc._lib.mcdc_workspace_bytes(ctypes.byref(d.d), ctypes.byref(mcdc.make_options()),
                                          ctypes.byref(n)) == 0
    plain = ctypes.c_size_t()
    d0 = mcdc._Desc(W.config2())
    assert mcdc._lib.mcdc_workspace_bytes(ctypes.byref(d0.d), ctypes.byref(mcdc.make_options()),
                                          ctypes.byref(plain)) == 0
    # three more arrays of 2 sides x 20 t x 60 x 60 bins (x, z in the plane y = 40)
    assert n.value - plain.value >= 3 * 8 * 2 * 20 * 60 * 60
    for bad in (dict(axis=3, pos=1.0), dict(axis=0, pos=float("nan"))):
        p["surface_tally"] = bad
        d = mcdc._Desc(p)
        assert mcdc._lib.mcdc_workspace_bytes(ctypes.byref(d.d), ctypes.byref(mcdc.make_options()),
                                              ctypes.byref(n)) == mcdc.E_INVALID
    assert np.isfinite(plain.value)


def test_every_declaration_names_its_source():
    """Each entry point of include/mcdc.h carries, in the comment right above
    it, a "Source:" line: the passage of the paper that defines what it
    computes, or what the call is for where the paper defines nothing."""
    src = open(HEADER).read()
    decl = re.compile(r"^(?:int|void|size_t|const char \*)\s*(mcdc_[a-z_0-9]+)\s*\(", re.M)
    prev_end = 0
    missing = []
    names = []
    for m in decl.finditer(src):
        names.append(m.group(1))
        block = src[prev_end:m.start()]
        comments = re.findall(r"/\*.*?\*/", block, flags=re.S)
        if not comments or "Source:" not in comments[-1]:
            missing.append(m.group(1))
        prev_end = src.index(";", m.end()) + 1
    assert set(names) == set(declared()), set(declared()) ^ set(names)
    assert not missing, missing
    # the paper-sourced calls name a section or figure of it
    for m in re.finditer(r"\n \* Source:(.*?)\*/", src, flags=re.S):
        text = " ".join(m.group(1).split())
        assert ("Sec." in text or "Fig." in text or "not in the paper" in text
                or text.startswith("as mcdc_") or "a reading" in text), text
