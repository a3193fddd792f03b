"""Build the gfx950 colour-LBM shared library (liblbm.so) in-tree with hipcc.

Run as ``python -m paper_2007_12266_amd.build``. Every HIP source is compiled for gfx950 with
packed-FP32 instruction selection disabled; the host-only pre-pass is compiled with g++.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_SOURCES = ["lbm_kernels.hip", "lbm_runtime.hip", "lbm_pool.hip", "lbm_morph.hip",
               "lbm_prep.hip", "lbm_transfer.hip"]
CPP_SOURCES = ["lbm_prepass.cpp"]
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include")]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-Wextra", "-I",
             os.path.join(ROOT, "include")]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True) -> str:
    """Compile every source (up to four compilers at a time) and link liblbm.so atomically;
    returns its path."""
    from concurrent.futures import ThreadPoolExecutor
    with tempfile.TemporaryDirectory(prefix="lbm_build_") as tmp:
        jobs = [["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o",
                 os.path.join(tmp, src + ".o")] for src in CPP_SOURCES]
        jobs += [[HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o",
                  os.path.join(tmp, src + ".o")] for src in HIP_SOURCES]
        objs = [cmd[-1] for cmd in jobs]
        with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as pool:
            for _ in pool.map(_run, jobs):   # re-raises the first failed compile
                pass
        out = os.path.join(tmp, "liblbm.so")
        _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", *objs, "-o", out])
        os.replace(out, LIB) if os.path.dirname(out) == os.path.dirname(LIB) else \
            _copy_atomic(out, LIB)
    return LIB


def _copy_atomic(src, dst):
    import shutil
    tmp = dst + ".tmp%d" % os.getpid()
    shutil.copyfile(src, tmp)
    os.replace(tmp, dst)


if __name__ == "__main__":
    build()
    print(LIB)
    sys.exit(0)
