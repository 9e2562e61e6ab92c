"""The library's host code (paper_1712_10279_amd/csrc/omt_api.cpp: validation,
step sizes, graph checks, eigenvalues, workspace layouts, the static entry
point's refusal, the matrix set-up) under AddressSanitizer, LeakSanitizer
and UndefinedBehaviorSanitizer.  Only the host side is instrumented (each
-fsanitize goes to the host compilation); the kernels come from the
library's ordinary build and are never launched, so this runs without a
GPU."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OBJ = os.path.join(ROOT, "_build", "obj")
CSRC = os.path.join(ROOT, "paper_1712_10279_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _kernel_objects():
    names = ["aux.o", "batch.o", "step3.o"] + [f"step_k{k}.o" for k in range(1, 10)]
    objs = [os.path.join(OBJ, n) for n in names]
    newest_src = max(os.path.getmtime(p) for p in glob.glob(os.path.join(CSRC, "*")))
    if not all(os.path.exists(o) and os.path.getmtime(o) >= newest_src for o in objs):
        from paper_1712_10279_amd import build
        build.build()
    return objs


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(HIPCC), reason="needs hipcc and g++")
def test_host_code_clean_under_sanitizers(tmp_path):
    api = tmp_path / "omt_api_san.o"
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN_HOST,
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", os.path.join(CSRC, "omt_api.cpp"), "-o", str(api)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    drv = tmp_path / "driver.o"
    r = subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-c",
                        os.path.join(ROOT, "tests", "csrc", "host_driver.cpp"), "-o", str(drv)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = tmp_path / "host_driver"
    r = subprocess.run(["g++", "-fsanitize=address,undefined", "-o", str(exe), str(drv), str(api),
                        *_kernel_objects(), "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64",
                        "-lrocprofiler-sdk-roctx"], capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available")
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", OMT_LOG="0")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-3000:]
    assert "0 failure(s)" in run.stdout
    assert "omt:" not in run.stderr
    # OMT_LOG=1: every refused call prints its status and detail on stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=dict(env, OMT_LOG="1"), timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-3000:]
    for line in ("omt: invalid argument: grid must be at least 2 x 2", "omt: invalid channel graph:",
                 "omt: step sizes violate the convergence condition:", "omt: workspace too small:"):
        assert line in run.stderr, line
