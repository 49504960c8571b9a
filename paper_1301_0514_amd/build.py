"""Build libscint.so (the gfx950 HIP library) in-tree with hipcc.

Usage: python -m paper_1301_0514_amd.build [--jobs N] [--verbose] [--incremental]

Compiles the row-pass kernel once per (precision, program), the auxiliary
kernels and the host C ABI, and links them into
paper_1301_0514_amd/lib/libscint.so.  Every call rebuilds from scratch unless
--incremental is given, which recompiles only the objects older than a source
they include (quoted #include files, followed recursively) or built with
other flags.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libscint.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAMS = ["ProgNoise", "ProgNoiseSwap", "ProgScreen", "ProgScreenProp", "ProgPhaseProp", "ProgPropIntensity",
            "ProgRealFwd", "ProgFwdRe", "ProgSmearMid", "ProgInvRe", "ProgVjpY", "ProgVjpX",
            "ProgPropField", "ProgVjpYField", "ProgApertureX", "ProgAbs2"]
# programs built for float only (their side transposes are complex64)
PROGRAMS_F32 = ["ProgNoiseT", "ProgNoiseSwapT", "ProgPhasePropT", "ProgPropIntensityT", "ProgRealFwdT", "ProgSmearMidT", "ProgInvReT"]

# gfx950 only; packed FP32 instructions are disabled (the compiler would
# otherwise form them from float code).
DEVICE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wno-unused-command-line-argument"]


def _jobs() -> list[tuple[list[str], str]]:
    jobs = []
    for real, is64 in (("float", 0), ("double", 1)):
        for prog in PROGRAMS + (PROGRAMS_F32 if not is64 else []):
            obj = os.path.join(BUILD, f"row_{real}_{prog}.o")
            cmd = [HIPCC, *DEVICE_FLAGS, f"-DSCINT_REAL={real}", f"-DSCINT_PROG={prog}",
                   f"-DSCINT_IS_F64={is64}", "-c", os.path.join(CSRC, "row_inst.hip"), "-o", obj]
            jobs.append((cmd, obj))
    for src in ("aux_kernels.hip", "scint_api.cpp", "twiddles.cpp"):
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        cmd = [HIPCC, *DEVICE_FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        jobs.append((cmd, obj))
    return jobs


def _deps(src: str, seen=None) -> set:
    """src and every file it includes with #include "...", recursively."""
    seen = set() if seen is None else seen
    src = os.path.normpath(src)
    if src in seen or not os.path.exists(src):
        return seen
    seen.add(src)
    with open(src, errors="replace") as fh:
        for name in re.findall(r'^\s*#\s*include\s+"([^"]+)"', fh.read(), flags=re.M):
            _deps(os.path.join(os.path.dirname(src), name), seen)
    return seen


def _up_to_date(cmd: list, obj: str) -> bool:
    stamp = obj + ".cmd"
    if not (os.path.exists(obj) and os.path.exists(stamp)):
        return False
    with open(stamp) as fh:
        if fh.read() != " ".join(cmd):
            return False
    src = cmd[cmd.index("-c") + 1]
    t = os.path.getmtime(obj)
    return all(os.path.getmtime(d) < t for d in _deps(src))


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    if jobs is None:
        jobs = int(os.environ.get("MAX_JOBS", "0")) or min(16, os.cpu_count() or 4)
    if not incremental:
        shutil.rmtree(BUILD, ignore_errors=True)
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    t0 = time.time()
    work = _jobs()

    def run(item):
        cmd, obj = item
        if incremental and _up_to_date(cmd, obj):
            return obj
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
        with open(obj + ".cmd", "w") as fh:
            fh.write(" ".join(cmd))
        if verbose:
            print("built", os.path.basename(obj), flush=True)
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(run, work))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("linked %s in %.1f s" % (LIB, time.time() - t0), flush=True)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--incremental", action="store_true")
    a = ap.parse_args(argv)
    build(a.jobs, a.verbose, a.incremental)
    return 0


if __name__ == "__main__":
    sys.exit(main())
