"""Build libfockhip.so in-tree with hipcc for gfx950.

    python paper_2111_00050_amd/build.py             # compile every unit, link
    python paper_2111_00050_amd/build.py --incremental

The fully unrolled stage kernel is instantiated once per (M, nrhs) in its
own translation unit (inst_stage.hip), the remaining kernels once per M
(inst_aux.hip), so that the large units compile in parallel.
build(incremental=True) recompiles only units older than the sources.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfockhip.so")
ARCH = os.environ.get("FH_OFFLOAD_ARCH", "gfx950")
MODES = list(range(1, 11))
NRHS = (1, 2, 4, 8, 16)

COMMON = [
    "-O3",
    "-std=c++20",
    f"--offload-arch={ARCH}",
    "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    # export only the C ABI (include/fockhip.h marks its declarations visible)
    "-fvisibility=hidden",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _units():
    """(source, object, extra flags, cost estimate) for every unit."""
    units = []
    for m in MODES:
        for r in NRHS:
            units.append((os.path.join(CSRC, "inst_stage.hip"), os.path.join(OBJ, f"stage_M{m}_R{r}.o"),
                          [f"-DFH_INST_M={m}", f"-DFH_INST_R={r}"], m ** 3 * (1 + r / 4)))
        units.append((os.path.join(CSRC, "inst_aux.hip"), os.path.join(OBJ, f"aux_M{m}.o"),
                      [f"-DFH_INST_M={m}"], m ** 3))
    for f in ("util.hip", "api.hip", "noalloc.hip", "derive.cpp"):
        src = os.path.join(CSRC, f)
        extra = ["-x", "hip"] if f.endswith(".cpp") else []
        units.append((src, os.path.join(OBJ, os.path.splitext(f)[0] + ".o"), extra, 1))
    return units


def _stale(src, obj):
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")]
    deps.append(os.path.join(HERE, "..", "include", "fockhip.h"))
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


def _compile(cc, src, obj, extra):
    cmd = [cc, *COMMON, *extra, "-c", src, "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{msgs}")
    return obj, time.time() - t0, msgs


def build(jobs: int | None = None, verbose: bool = True, incremental: bool = False) -> str:
    cc = hipcc()
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    units = _units()
    todo = [u for u in units if not incremental or _stale(u[0], u[1])]
    todo.sort(key=lambda u: -u[3])  # longest first
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, cc, *u[:3]) for u in todo]
        for f in cf.as_completed(futs):
            obj, dt, msgs = f.result()
            if verbose:
                print(f"[build] {os.path.basename(obj)} {dt:.1f}s", flush=True)
                if msgs.strip():
                    print(msgs, flush=True)
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *[u[1] for u in units]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"[build] {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--incremental", action="store_true")
    a = ap.parse_args()
    build(a.jobs, incremental=a.incremental)
    sys.exit(0)
