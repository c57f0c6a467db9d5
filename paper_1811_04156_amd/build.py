"""Builds librjpath.so (the gfx950 HIP library) in-tree with hipcc.

Each source compiles to its own object in parallel (the step-kernel variants
are split over several units for that reason), then the objects are linked
into one shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librjpath.so")
SOURCES = ["rj_run_f32.hip", "rj_run_f64.hip", "rj_run_f32_mala.hip", "rj_run_f64_mala.hip", "rj_run_f32_lmala.hip",
           "rj_run_f64_lmala.hip", "rj_run_f32_tree.hip", "rj_run_f64_tree.hip",
           "rj_sampler.hip", "rj_anchor.hip", "rj_stats.hip", "rj_noalloc.hip", "rj_observe.hip", "rj_api.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # contract a*b+c only inside one expression, so that inlined copies of the
    # same arithmetic round identically wherever they are used
    "-ffp-contract=on",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _jobs() -> int:
    try:
        n = int(os.environ.get("MAX_JOBS", "0"))
    except ValueError:
        n = 0
    return max(1, min(n or (os.cpu_count() or 1), 16, len(SOURCES)))


def build(verbose: bool = False, extra=None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(HERE, "..", "include")]
    with tempfile.TemporaryDirectory(prefix="rjpath_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[hipcc, *HIPCC_FLAGS, *(extra or []), *inc, "-c", "-o", o, os.path.join(CSRC, s)]
                for s, o in zip(SOURCES, objs)]

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd, capture_output=True, text=True)

        with ThreadPoolExecutor(_jobs()) as ex:
            results = list(ex.map(run, cmds))
        for r in results:
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError("hipcc failed building librjpath.so")
        tmp = LIB + ".tmp"
        r = run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking librjpath.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
