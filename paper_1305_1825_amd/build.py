"""Compile the HIP library libbhmc.so for gfx950 (in-tree).

Every translation unit is compiled with hipcc; the evaluation kernels are
compiled once per expansion order p = 0..10 so that the Taylor recurrence is
fully unrolled for that order.  Floating-point contraction is off so that the
decisions taken in floating point (keys, MAC, walls, overlaps) follow the
written left-to-right expressions; fused multiply-adds are written explicitly
where they are wanted.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libbhmc.so")
P_MAX = 10

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I" + INCLUDE, "-I" + CSRC,
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, obj: str, defines=()) -> str:
    cmd = [hipcc()] + HIPCC_FLAGS + ["-D%s" % d for d in defines] + ["-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), res.stdout, res.stderr))
    return obj


def build(jobs: int | None = None, verbose: bool = False, phase_timers: bool = False) -> str:
    """Compile every translation unit and link libbhmc.so (or, with phase_timers, the
    instrumented libbhmc_phase.so beside it); always recompiles."""
    build_dir = BUILD + ("_phase" if phase_timers else "")
    lib_path = os.path.join(HERE, "libbhmc_phase.so") if phase_timers else LIB
    extra = ("BHMC_PHASE_TIMERS",) if phase_timers else ()
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = [
        (os.path.join(CSRC, "bhmc_build.hip"), os.path.join(build_dir, "bhmc_build.o"), extra),
        (os.path.join(CSRC, "bhmc_api.hip"), os.path.join(build_dir, "bhmc_api.o"), extra),
    ]
    for p in range(P_MAX + 1):
        units.append((os.path.join(CSRC, "bhmc_eval.hip"), os.path.join(build_dir, "bhmc_eval_p%d.o" % p),
                      ("BHMC_P=%d" % p,) + extra))

    def order_of(u):
        ps = [d for d in u[2] if d.startswith("BHMC_P=")]
        return -int(ps[0].split("=")[1]) if ps else 0

    # the largest orders take longest: start them first
    units.sort(key=order_of)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(*u), units))
    tmp = lib_path + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (res.stdout, res.stderr))
    os.replace(tmp, lib_path)
    if verbose:
        print("built", lib_path)
    return lib_path


if __name__ == "__main__":
    build(verbose=True, phase_timers="--phase-timers" in sys.argv[1:])
    sys.exit(0)
