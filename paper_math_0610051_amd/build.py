"""Build the gfx950 HIP library libfio.so in-tree (paper_math_0610051_amd/_lib/).

Every device source is compiled by hipcc for gfx950 only; packed FP32
instructions are disabled (-packed-fp32-ops).  Host-only C++ is compiled by
g++.  Objects are built in parallel and linked with hipcc.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
OBJ_DIR = os.path.join(OUT_DIR, "obj")
LIB_PATH = os.path.join(OUT_DIR, "libfio.so")

HIP_SOURCES = ["abi.hip", "plan.hip", "apply.hip", "adjoint.hip", "multi.hip", "learned.hip", "autotune.hip",
               "taylor.hip"]
CXX_SOURCES = ["linalg.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-command-line-argument",
]
CXX_FLAGS = ["-O2", "-fPIC", "-std=c++17"]
LINK_LIBS = ["-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]  # rocBLAS: the Taylor factors' Gram and product GEMMs


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("command failed: %s\n%s" % (" ".join(cmd), p.stdout))
    return p.stdout


def source_digest() -> str:
    """SHA-256 (first 16 hex digits) of every file under csrc/: the build id
    that fio_version() reports and the autotuner keys its cache with."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        path = os.path.join(CSRC, name)
        if os.path.isfile(path):
            h.update(name.encode())
            with open(path, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every source (always) and link libfio.so; returns its path."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    cmds = []
    objs = []
    build_id = ["-DFIO_BUILD_ID=\"%s\"" % source_digest()]
    for src in HIP_SOURCES:
        obj = os.path.join(OBJ_DIR, src + ".o")
        cmds.append([HIPCC] + HIP_FLAGS + build_id + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in CXX_SOURCES:
        obj = os.path.join(OBJ_DIR, src + ".o")
        cmds.append(["g++"] + CXX_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                sys.stdout.write(out)
    tmp = LIB_PATH + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + LINK_LIBS)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def clean():
    shutil.rmtree(OUT_DIR, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose=True))
