"""Build ``libdgc.so`` in-tree for gfx950.

Host preprocessing (mesh build, coloring, layout, tables) is plain C++17
compiled with g++; the kernels and device entry points are HIP compiled with
hipcc for gfx950; the shared library is linked with hipcc.  Run as
``python -m paper_1601_07613_amd.build`` (or call :func:`build`).
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
OUT = PKG / "libdgc.so"
BUILD = PKG / "_build"
INCLUDE = PKG.parent / "include"

ARCH = os.environ.get("DGC_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", "g++")

HOST_SOURCES = sorted((CSRC / "host").glob("*.cpp"))
HIP_SOURCES = sorted((CSRC / "kernels").glob("*.hip"))

HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter", f"-I{INCLUDE}"]
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", f"-I{INCLUDE}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n%s\n%s%s" % (" ".join(map(str, cmd)), r.stdout, r.stderr))
    return r


def build(verbose: bool = False) -> Path:
    """Compile every source and link ``libdgc.so`` (always rebuilds)."""
    BUILD.mkdir(exist_ok=True)
    jobs = []
    for src in HOST_SOURCES:
        obj = BUILD / (src.stem + ".host.o")
        jobs.append([CXX, *HOST_FLAGS, "-c", str(src), "-o", str(obj)])
    for src in HIP_SOURCES:
        obj = BUILD / (src.stem + ".hip.o")
        jobs.append([HIPCC, *HIP_FLAGS, "-c", str(src), "-o", str(obj)])
    workers = min(len(jobs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout, r.stderr, file=sys.stderr)
    objs = [str(BUILD / (s.stem + ".host.o")) for s in HOST_SOURCES] + [
        str(BUILD / (s.stem + ".hip.o")) for s in HIP_SOURCES]
    tmp = OUT.with_suffix(".so.tmp")
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *objs])
    os.replace(tmp, OUT)
    return OUT


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
