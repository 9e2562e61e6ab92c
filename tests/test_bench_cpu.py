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
        files = tuple(e["sources"])
        assert files in (bench.STEP_SOURCES, bench.STEP3_SOURCES)
        rows = e.get("rows", 0)
        # reported for the source the counters were taken on, else null
        if e["kernel_sha"] != bench._kernel_hash(files):
            assert bench._traffic(key, rows, files) is None
            continue
        assert bench._traffic(key, rows, files) == e["bytes_per_launch"]
        # other shapes, sizes and kernels have no counters
        assert bench._traffic(key, (rows or 1) + 1, files) is None
        assert bench._traffic(key + "_other", rows, files) is None
        other = bench.STEP3_SOURCES if files == bench.STEP_SOURCES else bench.STEP_SOURCES
        assert bench._traffic(key, rows, other) is None
        # counted traffic is positive and within 1.5x of the launch's algorithmic bytes
        assert 0 < e["bytes_per_launch"] <= 1.5 * e["algorithmic_bytes"]


def test_iteration_caps_per_workload(monkeypatch):
    """Time-to-tolerance workloads stop at 3 million iterations unless told
    otherwise; the loss workload, whose slowest pair needs about 6.9 million
    to reach 1e-6, keeps 0 here and uses its own cap of 10 million."""
    for argv, cap in ((["--workload", "rgb"], 3_000_000), (["--workload", "batched"], 3_000_000),
                      (["--workload", "loss"], 0), (["--workload", "loss", "--cap", "500"], 500),
                      (["--workload", "rgb", "--cap", "7"], 7)):
        monkeypatch.setattr(sys, "argv", ["bench.py"] + argv)
        assert bench._parse().cap == cap, argv
