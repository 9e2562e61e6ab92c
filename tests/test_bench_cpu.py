"""Host-side behaviour of bench.py: the one-GPU contract and the rule that
counted HBM traffic is reported only for the kernel source and launch shape
it was measured on (profiles/traffic.json)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_only_for_the_profiled_source_and_shape():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        entries = json.load(fh)
    assert entries, "no counter summary committed"
    for key, e in entries.items():
        T, size = int(key.split("_")[0][1:]), int(key.split("_n")[1])
        # reported for the source the counters were taken on, else null
        if e["kernel_sha"] != bench._kernel_hash():
            assert bench._traffic(T, size, e.get("rows", 0)) is None
            continue
        assert bench._traffic(T, size, e.get("rows", 0)) == e["bytes_per_launch"]
        # other shapes and sizes have no counters
        assert bench._traffic(T, size, (e.get("rows") or 1) + 1) is None
        assert bench._traffic(T + 8, size) is None
        assert bench._traffic(T, size + 1) is None
        # counted traffic is positive and no more than the algorithmic bytes of T one-pass iterations
        assert 0 < e["bytes_per_launch"] <= (7 * 8 + 2 * 7) * 4 * size * size * T * 1.5
