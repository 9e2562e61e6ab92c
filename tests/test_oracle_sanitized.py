"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): any out-of-bounds access, leak or undefined operation on
small problems of every shape class fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "orc_san"
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-o", str(exe), os.path.join(ROOT, "oracle", "omt_oracle.c"),
           os.path.join(ROOT, "tests", "csrc", "oracle_sanitize_main.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available")
    assert r.returncode == 0, r.stderr
    # other libraries may be preloaded into every process; let ASan run after them
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stderr[-3000:]
    assert run.stdout.count("residual") == 12
