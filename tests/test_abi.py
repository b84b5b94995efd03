"""The C-ABI library loads on the CPU and exports every entry point that
include/mcdc.h declares (no compute calls: those need a GPU)."""
import ctypes
import os
import re

import pytest

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
