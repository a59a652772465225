"""Build the HIP library (libvrcube.so) in-tree for gfx950 with hipcc.

Each .hip file under csrc/ is compiled to an object in _build/ (in parallel),
then linked into paper_1012_2909_amd/libvrcube.so.  Packed-FP32 instructions
are disabled for device code.  build_all() also writes the debug library
libvrcube_debug.so (objects in _build_debug/, every source compiled with
VR_DEBUG_BOUNDS: index-range checks of the volume gathers and LDS boxes).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvrcube.so")
BUILD_DEBUG = os.path.join(HERE, "_build_debug")
LIB_DEBUG = os.path.join(HERE, "libvrcube_debug.so")
ARCH = os.environ.get("VR_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(os.path.dirname(HERE), "include")]


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    # keep warnings other than the host pass's note about the device-only feature
    err = "\n".join(line for line in r.stderr.splitlines() if "packed-fp32-ops" not in line and line.strip())
    if err:
        print(err, file=sys.stderr)
    return obj


def _link(objs, lib: str) -> str:
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


def build(jobs: int | None = None, csrc: str = CSRC, build_dir: str = BUILD, lib: str = LIB, extra=()) -> str:
    """Compile csrc/*.hip and link the shared library (by default the
    in-tree libvrcube.so; other directories and outputs build variants)."""
    os.makedirs(build_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(csrc, "*.hip")))
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, build_dir, extra), srcs))
    return _link(objs, lib)


def build_all(jobs: int | None = None) -> tuple[str, str]:
    """The release library and the debug (VR_DEBUG_BOUNDS) library, their
    compiles sharing one pool of jobs."""
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(BUILD_DEBUG, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(8, os.cpu_count() or 1)
    # the slowest sources first, so the pool's tail is short
    srcs.sort(key=lambda f: -os.path.getsize(f))
    tasks = [(f, BUILD, ()) for f in srcs] + [(f, BUILD_DEBUG, ("-DVR_DEBUG_BOUNDS",)) for f in srcs]
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda t: _compile(*t), tasks))
    names = sorted(os.path.basename(f) + ".o" for f in srcs)
    rel = _link([os.path.join(BUILD, n) for n in names], LIB)
    dbg = _link([os.path.join(BUILD_DEBUG, n) for n in names], LIB_DEBUG)
    return rel, dbg


if __name__ == "__main__":
    print(build_all())
