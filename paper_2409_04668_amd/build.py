"""Ahead-of-time build of libmcdc.so for gfx950 with hipcc.

Flags that matter for the method:
  -ffp-contract=off      no fused multiply-add contraction, so every FP64
                         expression rounds exactly as written;
  -munsafe-fp-atomics    FP64 atomic adds lower to the hardware
                         global_atomic_add_f64 / ds_add_f64 instructions;
  -packed-fp32-ops off   no packed FP32 instructions are generated.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmcdc.so")
SOURCES = ["mcdc_api.hip", "mcdc_history.hip", "mcdc_event.hip", "mcdc_mlp.hip", "mcdc_batch.hip",
           "mcdc_micro.hip", "mcdc_wwmap.hip", "mcdc_keff.hip"]
ARCH = os.environ.get("MCDC_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17", "-ffp-contract=off",
         "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _obj(src: str, outdir: str) -> str:
    return os.path.join(outdir, src.replace(".hip", ".o"))


def _compile(src: str, outdir: str, extra) -> str:
    obj = _obj(src, outdir)
    cmd = ["hipcc", "-c", *FLAGS, *extra, os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False, extra=()) -> str:
    outdir = os.path.join(HERE, "_build")
    os.makedirs(outdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(len(srcs), 6)) as ex:
        objs = list(ex.map(lambda s: _compile(s, outdir, list(extra)), srcs))
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
