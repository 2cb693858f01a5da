"""Build libpiso.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2505_16992_amd.build  [--jobs N] [--debug]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libpiso.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["piso_api.hip", "piso_fwd.hip", "piso_krylov.hip", "piso_mg.hip", "piso_line.hip", "piso_outflow.hip",
           "piso_stats.hip", "piso_bwd.hip", "piso_noalloc.hip",
           "piso_moments.hip", "piso_zmarch.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PISO_OFFLOAD_ARCH", "gfx950")

# packed FP32 instructions are disabled for all device code (see the design notes)
COMMON = [
    "--offload-arch=" + ARCH,
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
]


def _compile(src: str, opt: list) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *opt, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-8000:]))
    return obj


HOST_SOURCES = ["piso_topology.cpp"]   # plain C++ (no device code)
CXX = os.environ.get("CXX", "g++")


def _compile_host(src: str, opt: list) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [CXX, "-std=c++17", "-fPIC", "-Wall", *opt, "-I" + os.path.join(ROOT, "include"), "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("%s failed for %s:\n%s\n%s" % (CXX, src, " ".join(cmd), r.stderr[-8000:]))
    return obj


def build(jobs: int = 4, debug: bool = False) -> str:
    if not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found at %s" % HIPCC)
    os.makedirs(BUILD, exist_ok=True)
    opt = ["-O0", "-g"] if debug else ["-O3"]
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, opt), SOURCES))
        objs += list(ex.map(lambda s: _compile_host(s, opt), HOST_SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr[-8000:]))
    shutil.move(tmp, OUT)
    return OUT


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--debug", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.debug))


if __name__ == "__main__":
    sys.exit(main())
