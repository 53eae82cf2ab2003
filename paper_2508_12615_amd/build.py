"""Build libwipes.so (gfx950) from csrc/ with hipcc, in-tree.

Every HIP source is compiled for gfx950 only, with FP contraction off (the
kernels place every fused multiply-add explicitly, so forward and backward
evaluate the per-pair rule identically) and with packed-FP32 instructions
disabled.  The shared library lands next to this file.

Usage: python -m paper_2508_12615_amd.build [--debug]
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libwipes.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["api.hip", "pipeline.hip", "project.hip", "binning.hip", "sort.hip", "blend.hip", "project_bwd.hip",
           "graph.hip", "autotune.hip", "serve.hip", "adam.hip", "probe.hip", "deform.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result", "-I" + os.path.join(HERE, "..", "include")]


def _compile(src: str, debug: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + (["-g"] if debug else []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s%s" % (src, r.stdout, r.stderr))
    return obj


def build(debug: bool = False, verbose: bool = True) -> str:
    """Compile every source (always) and link libwipes.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, debug), srcs))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(debug="--debug" in sys.argv)
