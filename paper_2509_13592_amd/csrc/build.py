"""Build libbccb.so for gfx950 in-tree (next to the Python binding).

Usage: python -m paper_2509_13592_amd.csrc.build  (or call build()).
Compiles every translation unit with hipcc in parallel, then links.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(PKG, "libbccb.so")

SOURCES = ["kernels.hip", "resident.hip", "batch_kernels.hip", "batch_resident.hip", "learned_kernels.hip", "dense_kernels.hip", "noalloc.hip", "spaced_kernels.hip", "extract.hip", "passes_f64.hip",
           "plan_math.cpp", "embed_math.cpp", "spaced.cpp", "solve_f64.cpp", "api.cpp", "batch.cpp", "learned.cpp", "dense.cpp"]
# the pass kernels are compiled once per transform length (parallel build)
PASS_LENGTHS = [8, 16, 32, 64, 128, 256, 512, 1024]
# the single-scene cooperative solver: row lengths (each with column lengths 32..512)
RESIDENT_LENGTHS = [32, 64, 128, 256, 512]

ARCH = os.environ.get("BCCB_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{HERE}", "-Wall", "-Wno-unused-function"]
# Packed FP32 instructions are disabled for every HIP translation unit.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(job) -> str:
    src, extra, tag = job
    path = os.path.join(HERE, src)
    obj = os.path.join(OBJDIR, f"{src}{tag}.o")
    cmd = [hipcc(), *COMMON, *extra, *DEVICE, "-c", path, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [hipcc(), *COMMON, *extra, "-x", "hip", *DEVICE, "-c", path, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = [(f"passes_n.hip", [f"-DPASS_N={n}"], f".{n}") for n in reversed(PASS_LENGTHS)]
    jobs += [(f"resident_n.hip", [f"-DRES_N1={n}"], f".{n}") for n in reversed(RESIDENT_LENGTHS)]
    jobs += [(s, [], "") for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    workers = max(1, min(int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16, len(jobs)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, jobs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
