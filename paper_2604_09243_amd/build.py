"""Builds ``libsbr.so`` (HIP for gfx950) in-tree with hipcc.

Usage: ``python -m paper_2604_09243_amd.build`` (or ``build()`` from Python).
Each source is compiled to an object under ``_build/`` and the objects are
linked into ``paper_2604_09243_amd/libsbr.so``.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(ROOT, "_build", "sbr")
LIB = os.path.join(HERE, "libsbr.so")
SOURCES = ["api.cpp", "batch.cpp", "surrogate.cpp", "mesh_prep.cpp", "plan.cpp", "sah.cpp", "bvh4.cpp", "lbvh.hip", "trace.hip",
           "po.hip", "scene.hip", "mlp.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("SBR_OFFLOAD_ARCH", "gfx950")
# -ffp-contract=off: the float32 intersection/reflection arithmetic is rounded
# exactly as written (fused multiply-adds only where written explicitly).
# -packed-fp32-ops: no packed fp32 instructions are generated.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-x", "hip", "--offload-arch=" + ARCH, "-ffp-contract=off",
         "-fno-gpu-rdc", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-command-line-argument",
         "-I" + os.path.join(ROOT, "include")]


def _compile(src, verbose):
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose=False, jobs=None):
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 8)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
