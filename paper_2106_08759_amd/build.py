"""Build the HIP library libntrupkg.so in-tree for gfx950 (hipcc).

The library is several objects compiled in parallel and linked into one
shared library:
  ntrup_api.hip                      the C ABI (host code)
  ntrup_pipeline.hip  x 4            -DNTRUP_P=653|761|857|1277: the stage
                                     pipeline and single operations of one p
  ntrup_persist.hip   x 4            -DNTRUP_LPK=2|4 -DNTRUP_PMIXED=0|1: the
                                     persistent fused kernel
No device symbol is shared between objects (no relocatable device code).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libntrupkg.so")
# the vector-ALU issue-rate probe used by bench.py --calib-valu (not part of the KeyGen library)
CALIB_LIB = os.path.join(HERE, "libcalib.so")
OBJDIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # no packed FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

# (object name, source, defines)
UNITS = [("ntrup_api", "ntrup_api.hip", [])] + \
    [("ntrup_p%d" % p, "ntrup_pipeline.hip", ["-DNTRUP_P=%d" % p]) for p in (1277, 761, 857, 653)] + \
    [("ntrup_pers%d_%s" % (l, "mixed" if m else "single"), "ntrup_persist.hip",
      ["-DNTRUP_LPK=%d" % l, "-DNTRUP_PMIXED=%d" % m]) for m in (1, 0) for l in (2, 4)]


def _newest_source() -> float:
    t = 0.0
    for d in (CSRC, INCLUDE):
        for name in os.listdir(d):
            if name.endswith((".h", ".hip")):
                t = max(t, os.path.getmtime(os.path.join(d, name)))
    return t


def _compile(unit, extra, verbose, force, newest):
    name, src, defs = unit
    obj = os.path.join(OBJDIR, name + ".o")
    if not force and os.path.exists(obj) and os.path.getmtime(obj) > newest:
        return obj
    tmp = obj + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + defs + (extra or []) + ["-c", os.path.join(CSRC, src), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, obj)
    return obj


def build(verbose: bool = False, extra: list[str] | None = None, out: str = LIB, force: bool = True,
          jobs: int | None = None) -> str:
    """Compile every object (all of them when force, else only those older
    than a source) in parallel and link the library."""
    os.makedirs(OBJDIR, exist_ok=True)
    newest = _newest_source()
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, extra, verbose, force, newest), UNITS))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    if out == LIB:
        build_calib(verbose)
    return out


def build_calib(verbose: bool = False) -> str:
    tmp = CALIB_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-shared", os.path.join(CSRC, "calib_valu.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, CALIB_LIB)
    return CALIB_LIB


if __name__ == "__main__":
    args = sys.argv[1:]
    incremental = "--incremental" in args
    build(verbose=True, extra=[a for a in args if a != "--incremental"], force=not incremental)
