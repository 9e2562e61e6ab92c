"""Build ``libomt.so`` (the HIP kernels and the C ABI) for gfx950 in-tree.

Every translation unit is compiled with hipcc in parallel; the step kernel
source is compiled once per channel count.  Always rebuilds.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OBJ = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(HERE, "libomt.so")
ARCH = os.environ.get("OMT_OFFLOAD_ARCH", "gfx950")
KMAX = 9

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # keep every floating-point expression as written: the step kernel must
    # give bit-identical iterates for every blocking depth
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _units():
    units = []
    for k in range(1, KMAX + 1):
        units.append((os.path.join(CSRC, "step.hip"), os.path.join(OBJ, f"step_k{k}.o"), [f"-DOMT_K={k}"]))
    units.append((os.path.join(CSRC, "step3.hip"), os.path.join(OBJ, "step3.o"), []))
    units.append((os.path.join(CSRC, "aux.hip"), os.path.join(OBJ, "aux.o"), []))
    units.append((os.path.join(CSRC, "batch.hip"), os.path.join(OBJ, "batch.o"), []))
    units.append((os.path.join(CSRC, "omt_api.cpp"), os.path.join(OBJ, "omt_api.o"), ["-x", "hip"]))
    return [u for u in units if os.path.exists(u[0])]


def _compile(unit, verbose, defines=()):
    src, obj, extra = unit
    cmd = [HIPCC] + COMMON + [f"-D{d}" for d in defines] + extra + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {os.path.basename(obj)}:\n{r.stderr[-6000:]}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return obj, warn


def build(verbose: bool = False, jobs: int | None = None, defines=(), out: str | None = None) -> str:
    """Compile and link; ``defines`` are extra -D macros and ``out`` another
    library path (for variants built side by side)."""
    obj_dir = OBJ if not defines else OBJ + "_" + "_".join(d.replace("=", "") for d in defines)
    os.makedirs(obj_dir, exist_ok=True)
    units = [(src, os.path.join(obj_dir, os.path.basename(obj)), extra) for src, obj, extra in _units()]
    jobs = jobs or min(len(units), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        results = list(ex.map(lambda u: _compile(u, verbose, defines), units))
    for obj, warn in results:
        if warn and verbose:
            print(f"[{os.path.basename(obj)}] {warn}", flush=True)
    objs = [r[0] for r in results]
    lib = out or LIB
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", lib + ".tmp"] + objs + ["-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    import argparse
    import time
    ap = argparse.ArgumentParser()
    ap.add_argument("-v", action="store_true")
    ap.add_argument("-D", action="append", default=[], help="extra preprocessor macro NAME=VALUE (variant builds side by side)")
    ap.add_argument("-o", default=None, help="library path (default: the package's libomt.so)")
    args = ap.parse_args()
    t0 = time.time()
    path = build(verbose=args.v, defines=args.D, out=args.o)
    print(f"built {path} in {time.time() - t0:.1f} s")
